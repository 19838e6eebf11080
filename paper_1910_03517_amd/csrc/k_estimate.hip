// Estimate and table kernels of section 3.1: one thread per (camera, side,
// block, channel) for the affine fit, one workgroup per (camera, side, block)
// for the tables, one thread per column for the blend weights.
#include "dev_estimate.h"
#include "dev_stats.h"

namespace rc {

__global__ __launch_bounds__(kThreads) void k_estimate(Geo g, Bufs b) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < g.n_cams * 2 * g.n_blocks * kCS && cam_active(g, u / (2 * g.n_blocks * kCS))) estimate_unit(g, b, u);
}

__global__ __launch_bounds__(kThreads) void k_build_lut(Geo g, Bufs b) {
  if (!cam_active(g, blockIdx.x / (2 * g.n_blocks))) return;
  lut_entry(g, b, blockIdx.x, threadIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_weights(Geo g, Bufs b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)g.n_cams * g.w_max) return;
  const int k = (int)(i / g.w_max);
  const int col = (int)(i - (int64_t)k * g.w_max);
  if (cam_active(g, k)) b.weights[i] = (uint16_t)blend_weight(g.cams[k].width, col);
}

// Estimate, tables and weights of one (camera, side, block) per workgroup:
// threads 0..2 fit the three channels, then every thread builds one table
// entry.  Workgroups of side 0, block 0 also write their camera's weights.
__global__ __launch_bounds__(kThreads) void k_estimate_lut(Geo g, Bufs b) {
  const int u3 = blockIdx.x;                 // (k * 2 + s) * nb + j
  const int tid = threadIdx.x;
  const int nb = g.n_blocks;
  const int k = u3 / (2 * nb);
  // Clear the whole-frame statistics that the apply pass of this frame-set
  // accumulates (skipped when the caller clears them itself).
  if (b.whole_hist) zero_whole(g, b, blockIdx.x * kThreads + tid, gridDim.x * kThreads);
  if (!cam_active(g, k)) return;
  if (tid < kCS) estimate_unit(g, b, u3 * kCS + tid);
  __syncthreads();
  lut_entry(g, b, u3, tid);
  if (u3 % (2 * nb) == 0)
    for (int col = tid; col < g.w_max; col += kThreads)
      b.weights[(int64_t)k * g.w_max + col] = (uint16_t)blend_weight(g.cams[k].width, col);
}

hipError_t launch_estimate_lut(const Geo& g, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_estimate_lut, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, b);
  return hipGetLastError();
}

hipError_t launch_estimate(const Geo& g, const Bufs& b, hipStream_t st) {
  const int total = g.n_cams * 2 * g.n_blocks * kCS;
  hipLaunchKernelGGL(k_estimate, dim3((total + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, b);
  return hipGetLastError();
}

hipError_t launch_build_lut(const Geo& g, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_build_lut, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)g.n_cams * g.w_max;
  hipLaunchKernelGGL(k_weights, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace rc
