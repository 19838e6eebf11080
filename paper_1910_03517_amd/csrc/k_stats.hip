// Statistics kernels: band statistics of section 3.1 (one workgroup per
// (camera, side, block)) and the clearing of the whole-frame statistics.
#include "dev_stats.h"

namespace rc {

__global__ __launch_bounds__(kThreads) void k_band_stats(Geo g, FramePtrs fp, Bufs b) {
  __shared__ StatsLds L;
  band_unit_dispatch(g, fp, b, blockIdx.x, L);
}

__global__ __launch_bounds__(kThreads) void k_zero_whole(Geo g, Bufs b) {
  zero_whole(g, b, blockIdx.x * kThreads + threadIdx.x, gridDim.x * kThreads);
}

hipError_t launch_band_stats(const Geo& g, const FramePtrs& fp, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_band_stats, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, fp, b);
  return hipGetLastError();
}

hipError_t launch_zero_whole(const Geo& g, const Bufs& b, hipStream_t st) {
  const int n = g.n_cams * kCS * kNB;
  hipLaunchKernelGGL(k_zero_whole, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace rc
