// Difference approach of section 3.3's attention mechanisms: the absolute
// difference of two consecutive frames, thresholded (a pixel is on when the
// difference exceeds tau << (bit_depth - 8) on some channel), counted per
// cell of c x c pixels, then summed over every window of m x m cells; a
// window is selected when its count exceeds theta.  Exact integers.
//
// k_diff_cells: one workgroup per (camera, cell row).  A thread takes groups
// of 4 consecutive pixels of the cell row's rows (c is a multiple of 4, so a
// group lies in one cell), counts its on-pixels over the c rows and adds the
// count to its cell in LDS; the cell row is then written out.  Both frames
// are read once: 2 x (samples x bytes) per pixel.
// k_windows: one thread per window, the m x m cell counts summed directly.
// Outputs are laid out over the largest camera's grid; entries beyond a
// camera's own cells or windows are written as zero (not selected).
#include "dev_apply.h"

namespace rc {

struct AttnArgs {
  const uint8_t* prev[RT_MAX_CAMS];
  uint32_t* cells;      // [K][hc][wc]
  uint32_t* windows;    // [K][hc - m + 1][wc - m + 1] or null
  uint8_t* selected;    // same shape or null
  int32_t hc, wc;       // padded cell grid of every camera
  int32_t cell, m;
  uint32_t tau, theta;  // tau in 8-bit units
};

constexpr int kAttnMaxCells = 32768 / 4;   // cells of one cell row for the widest frame and c = 4

struct AttnLds {
  uint32_t cnt[kAttnMaxCells];
};

// On-pixels among the npx pixels (1..4) of a group starting at byte off.
template <int C, int BPS>
__device__ inline uint32_t group_on(__amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb, int off, int npx,
                                    uint32_t thr) {
  constexpr int NW = C * BPS;
  uint32_t on = 0;
  if (npx == 4) {
    uint32_t a[NW], b[NW];
    load_group<NW, 0>(ra, off, a);
    load_group<NW, 0>(rb, off, b);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      uint32_t d = 0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int i = p * C + c;
        uint32_t x, y;
        if (BPS == 1) { x = (a[i >> 2] >> (8 * (i & 3))) & 0xffu; y = (b[i >> 2] >> (8 * (i & 3))) & 0xffu; }
        else { x = (a[i >> 1] >> (16 * (i & 1))) & 0xffffu; y = (b[i >> 1] >> (16 * (i & 1))) & 0xffffu; }
        const uint32_t e = x > y ? x - y : y - x;
        d = d > e ? d : e;
      }
      on += d > thr;
    }
  } else {
    for (int p = 0; p < npx; ++p) {
      uint32_t d = 0;
      for (int c = 0; c < C; ++c) {
        const int o = off + (p * C + c) * BPS;
        uint32_t x, y;
        if (BPS == 1) { x = __builtin_amdgcn_raw_buffer_load_b8(ra, o, 0, 0); y = __builtin_amdgcn_raw_buffer_load_b8(rb, o, 0, 0); }
        else { x = __builtin_amdgcn_raw_buffer_load_b16(ra, o, 0, 0); y = __builtin_amdgcn_raw_buffer_load_b16(rb, o, 0, 0); }
        const uint32_t e = x > y ? x - y : y - x;
        d = d > e ? d : e;
      }
      on += d > thr;
    }
  }
  return on;
}

template <int C, int BPS>
__device__ void diff_cell_row(const DevCam& cam, const FramePtrs& fp, const AttnArgs& a, int k, int ci,
                              AttnLds& L) {
  const int tid = threadIdx.x;
  const int W = cam.width, H = cam.height, c = a.cell;
  const int ncell = (W + c - 1) / c;
  for (int i = tid; i < ncell; i += kThreads) L.cnt[i] = 0;
  __syncthreads();
  const __amdgpu_buffer_rsrc_t ra = frame_rsrc(fp.in[k], cam);
  const __amdgpu_buffer_rsrc_t rb = frame_rsrc(a.prev[k], cam);
  const uint32_t thr = a.tau << (cam.bit_depth - 8);
  const int pitch = (int)cam.pitch;
  const int r0 = ci * c, r1 = min(H, r0 + c);
  const int ngroups = (W + 3) >> 2;
  for (int g = tid; g < ngroups; g += kThreads) {
    const int col0 = g * 4, npx = min(4, W - col0);
    uint32_t n = 0;
    for (int r = r0; r < r1; ++r) n += group_on<C, BPS>(ra, rb, r * pitch + col0 * C * BPS, npx, thr);
    if (n) atomicAdd(&L.cnt[col0 / c], n);
  }
  __syncthreads();
  uint32_t* out = a.cells + ((int64_t)k * a.hc + ci) * a.wc;
  for (int i = tid; i < a.wc; i += kThreads) out[i] = i < ncell ? L.cnt[i] : 0u;
}

__global__ __launch_bounds__(kThreads) void k_diff_cells(Geo g, FramePtrs fp, AttnArgs a) {
  __shared__ AttnLds L;
  const int k = blockIdx.y, ci = blockIdx.x;
  if (!cam_active(g, k)) return;
  const DevCam cam = uniform_cam(g.cams[k]);
  if (ci * a.cell >= cam.height) {   // below the camera's cell grid: zeros
    uint32_t* out = a.cells + ((int64_t)k * a.hc + ci) * a.wc;
    for (int i = threadIdx.x; i < a.wc; i += kThreads) out[i] = 0u;
    return;
  }
  if (cam.bps == 2) diff_cell_row<1, 2>(cam, fp, a, k, ci, L);
  else if (cam.channels == 3) diff_cell_row<3, 1>(cam, fp, a, k, ci, L);
  else diff_cell_row<1, 1>(cam, fp, a, k, ci, L);
}

__global__ __launch_bounds__(kThreads) void k_windows(Geo g, AttnArgs a) {
  const int k = blockIdx.y;
  if (!cam_active(g, k)) return;
  const int hw = a.hc - a.m + 1, ww = a.wc - a.m + 1;
  const int w = blockIdx.x * kThreads + threadIdx.x;
  if (w >= hw * ww) return;
  const int wy = w / ww, wx = w - (w / ww) * ww;
  // Windows of this camera's own cell grid; the rest of the padded grid is 0.
  const int hck = (g.cams[k].height + a.cell - 1) / a.cell, wck = (g.cams[k].width + a.cell - 1) / a.cell;
  const uint32_t* cells = a.cells + (int64_t)k * a.hc * a.wc;
  uint32_t s = 0;
  const bool inside = wy + a.m <= hck && wx + a.m <= wck;
  if (inside)
    for (int dy = 0; dy < a.m; ++dy)
      for (int dx = 0; dx < a.m; ++dx) s += cells[(wy + dy) * a.wc + wx + dx];
  const int64_t o = (int64_t)k * hw * ww + w;
  if (a.windows) a.windows[o] = s;
  if (a.selected) a.selected[o] = inside && s > a.theta ? 1 : 0;
}

hipError_t launch_attention(const Geo& g, const FramePtrs& fp, const uint8_t* const* prev, uint32_t* cells,
                            uint32_t* windows, uint8_t* selected, int hc, int wc, int cell, int m, uint32_t tau,
                            uint32_t theta, hipStream_t st) {
  AttnArgs a{};
  for (int k = 0; k < g.n_cams; ++k) a.prev[k] = prev[k];
  a.cells = cells;
  a.windows = windows;
  a.selected = selected;
  a.hc = hc;
  a.wc = wc;
  a.cell = cell;
  a.m = m;
  a.tau = tau;
  a.theta = theta;
  hipLaunchKernelGGL(k_diff_cells, dim3(hc, g.n_cams), dim3(kThreads), 0, st, g, fp, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nw = (hc - m + 1) * (wc - m + 1);
  if (nw > 0 && (windows || selected)) {
    hipLaunchKernelGGL(k_windows, dim3((nw + kThreads - 1) / kThreads, g.n_cams), dim3(kThreads), 0, st, g, a);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace rc
