// Apply kernel of section 3.1, weights read from the caller's table.  With
// statistics, each tile adds its input histogram and sums to the camera's
// whole-frame statistics with atomics.
#include "dev_apply.h"

namespace rc {

// Workgroups stride over the tiles (one tile each when the grid equals the
// tile count).  Tiles are independent: no workgroup waits for another.
#ifndef RC_APPLY_WAVES
#define RC_APPLY_WAVES 1
#endif
template <bool WRITE, bool STATS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(RC_APPLY_WAVES)))
void k_apply(Geo g, FramePtrs fp, Bufs b) {
  __shared__ ApplyLds L;
  for (int ti = blockIdx.x; ti < g.n_tiles; ti += gridDim.x) {
    if (!cam_active(g, g.tiles[ti].cam)) continue;   // uniform over the workgroup
    apply_tile_dispatch<WRITE, STATS, true>(g, fp, b, ti, L);
    __syncthreads();
  }
}

hipError_t launch_apply(const Geo& g, const FramePtrs& fp, const Bufs& b, bool write, bool stats, hipStream_t st) {
  const int n = (g.apply_grid > 0 && g.apply_grid < g.n_tiles) ? g.apply_grid : g.n_tiles;
  const dim3 grid(n), block(kThreads);
  if (write && stats) hipLaunchKernelGGL((k_apply<true, true>), grid, block, 0, st, g, fp, b);
  else if (write) hipLaunchKernelGGL((k_apply<true, false>), grid, block, 0, st, g, fp, b);
  else if (stats) hipLaunchKernelGGL((k_apply<false, true>), grid, block, 0, st, g, fp, b);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace rc
