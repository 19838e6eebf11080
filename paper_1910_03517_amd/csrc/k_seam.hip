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
// An item is (camera, kind): kind 0 the seam at the camera's right side (its
// facing camera as the right image), kind 1 the interior seam at column
// floor(W/2).  k_seam_rows: one workgroup per (item, chunk of 64 image rows):
// thread (row, box) sums the f x C samples of its box's part of one image
// row, exact integers; the f partial sums of each box meet in LDS, and one
// thread per box row evaluates the row value in binary64 with the operation
// order of the definition (box means as sum / f^2, the two differences,
// their difference, squares summed over the channels in order, one square
// root per norm) and writes it to the row buffer.  k_seam_mean: one
// workgroup per item; thread t sums a contiguous range of rows in row order,
// then one thread adds the 256 partial sums in thread order and divides by
// the row count: deterministic.
#include "dev_common.h"

namespace rc {

constexpr int kSeamChunk = kThreads / 4;   // image rows per workgroup of k_seam_rows

struct SeamArgs {
  double* seam;        // [K]
  double* interior;    // [K]
  double* rows;        // [K][2][row_stride]
  int32_t row_stride;
  int32_t factor;
};

// Geometry of one item: right-image camera, first columns of the left and
// right box pairs, and the number of box rows (0 = undefined).
struct SeamItem {
  int kr, xl, xr, n;
};

__device__ inline SeamItem seam_item(const Geo& g, int k, int kind, int f) {
  const DevCam& cl = g.cams[k];
  SeamItem it{kind == 0 ? cl.face_cam[1] : k, 0, 0, 0};
  if (it.kr < 0) return it;
  const DevCam& cr = g.cams[it.kr];
  if (kind == 0) {
    it.xl = cl.width - 2 * f;
    if (cl.width >= 2 * f && cr.width >= 2 * f) it.n = min(cl.height, cr.height) / f;
  } else {
    const int m = cl.width / 2;
    it.xl = m - 2 * f;
    it.xr = m;
    if (m >= 2 * f && cl.width - m >= 2 * f) it.n = cl.height / f;
  }
  return it;
}

// Sum of each channel over columns [x0, x0 + f) of one image row.
template <int C, int BPS>
__device__ inline void row_box_sums(__amdgpu_buffer_rsrc_t r, int64_t pitch, int y, int x0, int f, int32_t (&s)[kCS]) {
#pragma unroll
  for (int c = 0; c < kCS; ++c) s[c] = 0;
  const int base = (int)((int64_t)y * pitch) + x0 * C * BPS;
  for (int x = 0; x < f; ++x) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int off = base + (x * C + c) * BPS;
      s[c] += BPS == 1 ? (int32_t)__builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0)
                       : (int32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    }
  }
}

struct SeamLds {
  int32_t part[kSeamChunk][4][kCS];     // per image row: box-column sums
  int64_t box[kSeamChunk][4][kCS];      // per box row: box sums
};

template <int C, int BPS>
__device__ void seam_rows_chunk(const Geo& g, const FramePtrs& fp, const SeamArgs& a, int k, int kind, int chunk,
                                SeamLds& L) {
  const int tid = threadIdx.x, f = a.factor;
  const SeamItem it = seam_item(g, k, kind, f);
  const int R = kSeamChunk / f;                 // box rows per chunk
  const int j0 = chunk * R;                     // first box row of the chunk
  if (it.n == 0 || j0 >= it.n) return;          // uniform over the workgroup
  const DevCam cl = uniform_cam(g.cams[k]);
  const DevCam cr = uniform_cam(g.cams[it.kr]);
  const int i = tid >> 2, b = tid & 3;          // image row in the chunk; box 0 = I-_{-1}, 1 = I-_0, 2 = I+_0, 3 = I+_1
  const int nrow = min(R, it.n - j0) * f;
  if (i < nrow) {
    int32_t s[kCS];
    const int y = j0 * f + i;
    if (b < 2) row_box_sums<C, BPS>(frame_rsrc(fp.in[k], cl), cl.pitch, y, it.xl + b * f, f, s);
    else row_box_sums<C, BPS>(frame_rsrc(fp.in[it.kr], cr), cr.pitch, y, it.xr + (b - 2) * f, f, s);
#pragma unroll
    for (int c = 0; c < kCS; ++c) L.part[i][b][c] = s[c];
  }
  __syncthreads();
  const int nbox = nrow / f;
  for (int t = tid; t < nbox * 4 * C; t += kThreads) {
    const int c = t % C, bb = (t / C) & 3, jj = t / (4 * C);
    int64_t s = 0;
    for (int r = 0; r < f; ++r) s += L.part[jj * f + r][bb][c];
    L.box[jj][bb][c] = s;
  }
  __syncthreads();
  if (tid < nbox) {
    const double area = (double)f * (double)f;
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
    a.rows[((int64_t)k * 2 + kind) * a.row_stride + j0 + tid] = (__builtin_sqrt(dp) + __builtin_sqrt(dm)) / 2.0;
  }
}

__global__ __launch_bounds__(kThreads) void k_seam_rows(Geo g, FramePtrs fp, SeamArgs a) {
  __shared__ SeamLds L;
  const int k = blockIdx.x >> 1, kind = blockIdx.x & 1;
  if (!cam_active(g, k)) return;
  const DevCam c = uniform_cam(g.cams[k]);
  if (c.bps == 2) seam_rows_chunk<1, 2>(g, fp, a, k, kind, blockIdx.y, L);
  else if (c.channels == 3) seam_rows_chunk<3, 1>(g, fp, a, k, kind, blockIdx.y, L);
  else seam_rows_chunk<1, 1>(g, fp, a, k, kind, blockIdx.y, L);
}

__global__ __launch_bounds__(kThreads) void k_seam_mean(Geo g, SeamArgs a) {
  __shared__ double part[kThreads];
  const int k = blockIdx.x >> 1, kind = blockIdx.x & 1;
  if (!cam_active(g, k)) return;
  const int tid = threadIdx.x;
  const int n = seam_item(g, k, kind, a.factor).n;
  double* out = kind == 0 ? a.seam : a.interior;
  if (n == 0) {
    if (tid == 0) out[k] = __builtin_nan("");
    return;
  }
  const double* rows = a.rows + ((int64_t)k * 2 + kind) * a.row_stride;
  const int per = (n + kThreads - 1) / kThreads;
  double s = 0.0;
  for (int i = tid * per; i < min(n, (tid + 1) * per); ++i) s = s + rows[i];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < kThreads; ++i) t = t + part[i];
    out[k] = t / (double)n;
  }
}

hipError_t launch_seam_cost(const Geo& g, const FramePtrs& fp, double* seam, double* interior, double* rows,
                            int row_stride, int factor, int max_rows, hipStream_t st) {
  const SeamArgs a{seam, interior, rows, row_stride, factor};
  const int per = kSeamChunk / factor;
  const int chunks = max(1, (max_rows + per - 1) / per);
  hipLaunchKernelGGL(k_seam_rows, dim3(g.n_cams * 2, chunks), dim3(kThreads), 0, st, g, fp, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seam_mean, dim3(g.n_cams * 2), dim3(kThreads), 0, st, g, a);
  return hipGetLastError();
}

}  // namespace rc
