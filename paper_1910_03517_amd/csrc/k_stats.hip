// Statistics kernels: band statistics of section 3.1 (one workgroup per
// (camera, side, block)) and the whole-frame reduction (one workgroup per
// camera) of the per-tile histograms left by the apply pass.
#include "dev_stats.h"

namespace rc {

__global__ __launch_bounds__(kThreads) void k_band_stats(Geo g, FramePtrs fp, Bufs b) {
  __shared__ StatsLds L;
  band_unit_dispatch(g, fp, b, blockIdx.x, L);
}

__global__ __launch_bounds__(kThreads) void k_whole_reduce(Geo g, Bufs b) {
  __shared__ StatsLds L;
  whole_reduce_cam(g, b, blockIdx.x, L);
}

hipError_t launch_band_stats(const Geo& g, const FramePtrs& fp, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_band_stats, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, fp, b);
  return hipGetLastError();
}

hipError_t launch_whole_reduce(const Geo& g, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_whole_reduce, dim3(g.n_cams), dim3(kThreads), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace rc
