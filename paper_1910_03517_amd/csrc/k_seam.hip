// Seam gradient cost of section 4.2 (the gradient-cost equation) on the
// device, as a monitor that can run on any frame-set (input or corrected).
//
// Frames are box-downsampled by `factor` in both directions.  For row i of a
// seam between a left image I- and a right image I+, with I-_{-1}, I-_0 the
// last two box columns of I- and I+_0, I+_1 the first two of I+,
//   d+_i = |(I+_1 - I+_0) - (I+_0 - I-_0)|,  d-_i = |(I-_{-1} - I-_0) - (I-_0 - I+_0)|,
// |.| the Euclidean norm over the channels in sample units; the cost is the
// mean over rows of (d+_i + d-_i) / 2.  The interior reference of the same
// section is the cost at a virtual seam in the middle of one image.
//
// One workgroup per (camera, kind): kind 0 the seam at the camera's right
// side (its facing camera as the right image), kind 1 the interior seam at
// column floor(W/2).  Thread t takes box (t % 4) of box rows t / 4, t / 4 +
// 64, ...: its f x f x C samples summed in exact integers; the four boxes of a
// row meet in LDS, and one thread per row evaluates the row value in binary64
// with the operation order of the definition above (box means as sum / f^2,
// the two differences, their difference, squares summed over the channels in
// order, one square root per norm).  The mean sums each thread's rows in row
// order and then the 64 partial sums in thread order: deterministic.
#include "dev_common.h"

namespace rc {

constexpr int kSeamRows = kThreads / 4;   // box rows per pass of a workgroup

struct SeamArgs {
  double* seam;        // [K]
  double* interior;    // [K]
  double* rows;        // [K][2][row_stride] or null
  int32_t row_stride;
  int32_t factor;
};

struct SeamLds {
  int64_t box[kSeamRows][4][kCS];
  double part[kSeamRows];
};

// Sum of each channel over rows [r0, r0 + f) and columns [c0, c0 + f).
template <int C, int BPS>
__device__ inline void box_sums(__amdgpu_buffer_rsrc_t r, int64_t pitch, int r0, int c0, int f, int64_t (&s)[kCS]) {
#pragma unroll
  for (int c = 0; c < kCS; ++c) s[c] = 0;
  for (int y = r0; y < r0 + f; ++y) {
    const int base = (int)((int64_t)y * pitch) + c0 * C * BPS;
    for (int x = 0; x < f; ++x) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int off = base + (x * C + c) * BPS;
        const uint32_t v = BPS == 1 ? __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0)
                                    : __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        s[c] += v;
      }
    }
  }
}

template <int C, int BPS>
__device__ void seam_item(const Geo& g, const FramePtrs& fp, const SeamArgs& a, int k, int kind, SeamLds& L) {
  const int tid = threadIdx.x;
  const int f = a.factor;
  const DevCam cl = uniform_cam(g.cams[k]);
  double* out = kind == 0 ? a.seam : a.interior;
  const int kr = kind == 0 ? cl.face_cam[1] : k;
  double* rows = a.rows ? a.rows + ((int64_t)k * 2 + kind) * a.row_stride : nullptr;
  int n = 0, xl = 0, xr = 0;   // box rows; first column of the left and of the right box pair
  DevCam cr = cl;
  if (kr >= 0) {
    cr = uniform_cam(g.cams[kr]);
    if (kind == 0) {
      xl = cl.width - 2 * f;
      xr = 0;
      if (cl.width >= 2 * f && cr.width >= 2 * f) n = min(cl.height, cr.height) / f;
    } else {
      const int m = cl.width / 2;
      xl = m - 2 * f;
      xr = m;
      if (m >= 2 * f && cl.width - m >= 2 * f) n = cl.height / f;
    }
  }
  if (n == 0) {
    if (tid == 0) out[k] = __builtin_nan("");
    return;
  }
  const __amdgpu_buffer_rsrc_t rl = frame_rsrc(fp.in[k], cl);
  const __amdgpu_buffer_rsrc_t rr = frame_rsrc(fp.in[kr], cr);
  const int b = tid & 3;          // box: 0 = I-_{-1}, 1 = I-_0, 2 = I+_0, 3 = I+_1
  const int lr = tid >> 2;        // box row within a pass
  const double area = (double)f * (double)f;
  double part = 0.0;
  for (int i0 = 0; i0 < n; i0 += kSeamRows) {
    const int i = i0 + lr;
    if (i < n) {
      int64_t s[kCS];
      if (b < 2) box_sums<C, BPS>(rl, cl.pitch, i * f, xl + b * f, f, s);
      else box_sums<C, BPS>(rr, cr.pitch, i * f, xr + (b - 2) * f, f, s);
#pragma unroll
      for (int c = 0; c < kCS; ++c) L.box[lr][b][c] = s[c];
    }
    __syncthreads();
    if (tid < kSeamRows && i0 + tid < n) {
      double dp = 0.0, dm = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double im1 = (double)L.box[tid][0][c] / area, im0 = (double)L.box[tid][1][c] / area;
        const double ip0 = (double)L.box[tid][2][c] / area, ip1 = (double)L.box[tid][3][c] / area;
        const double tp = (ip1 - ip0) - (ip0 - im0);
        const double tm = (im1 - im0) - (im0 - ip0);
        dp = dp + tp * tp;
        dm = dm + tm * tm;
      }
      const double v = (__builtin_sqrt(dp) + __builtin_sqrt(dm)) / 2.0;
      if (rows) rows[i0 + tid] = v;
      part = part + v;
    }
    __syncthreads();
  }
  if (tid < kSeamRows) L.part[tid] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int t = 0; t < kSeamRows; ++t) s = s + L.part[t];
    out[k] = s / (double)n;
  }
}

__global__ __launch_bounds__(kThreads) void k_seam_cost(Geo g, FramePtrs fp, SeamArgs a) {
  __shared__ SeamLds L;
  const int k = blockIdx.x >> 1, kind = blockIdx.x & 1;
  if (!cam_active(g, k)) return;
  const DevCam c = uniform_cam(g.cams[k]);
  if (c.bps == 2) seam_item<1, 2>(g, fp, a, k, kind, L);
  else if (c.channels == 3) seam_item<3, 1>(g, fp, a, k, kind, L);
  else seam_item<1, 1>(g, fp, a, k, kind, L);
}

hipError_t launch_seam_cost(const Geo& g, const FramePtrs& fp, double* seam, double* interior, double* rows,
                            int row_stride, int factor, hipStream_t st) {
  const SeamArgs a{seam, interior, rows, row_stride, factor};
  hipLaunchKernelGGL(k_seam_cost, dim3(g.n_cams * 2), dim3(kThreads), 0, st, g, fp, a);
  return hipGetLastError();
}

}  // namespace rc
