// Apply kernel of section 3.1, weights read from the caller's table.  With
// statistics, each tile adds its input histogram and sums to the camera's
// whole-frame statistics with atomics.
#include <hip/hip_ext.h>

#include "dev_apply.h"

namespace rc {

// Workgroup w takes its run of segments (one tile, or a contiguous share of
// all rows balanced by bytes); the histogram of a camera stays in LDS across
// the run's segments of that camera and is added to the whole-frame
// statistics once, after its last one.  No workgroup waits for another.
#ifndef RC_APPLY_WAVES
#define RC_APPLY_WAVES 1
#endif
// VBLEND: the maps of adjacent blocks blended row by row (a kernel of its own,
// so that its registers do not weigh on the plain pass).
template <bool WRITE, bool STATS, bool VBLEND>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(RC_APPLY_WAVES)))
void k_apply(Geo g, FramePtrs fp, Bufs b) {
  __shared__ ApplyLds L;
  const int s0 = uniform(g.wg_seg[blockIdx.x]), s1 = uniform(g.wg_seg[blockIdx.x + 1]);
  int prev = -1;
  for (int s = s0; s < s1;) {
    const int cam = uniform(g.tiles[s].cam);
    if (!cam_active(g, cam)) {   // uniform over the workgroup
      ++s;
      continue;
    }
    s = apply_tile_dispatch<WRITE, STATS, true, VBLEND>(g, fp, b, s, s1, L, cam != prev);
    __syncthreads();
    prev = cam;
  }
}

// Apply with statistics of several frame-sets of the rig (see SetPtrs): the
// same runs of segments as k_apply, once per set, set-major, so that one
// launch has no drain between the frame-sets it holds.
template <bool VBLEND>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(RC_APPLY_WAVES)))
void k_apply_sets(Geo g, SetPtrs sp) {
  __shared__ ApplyLds L;
  const int f = (int)blockIdx.x / g.n_wg, w = (int)blockIdx.x - f * g.n_wg;
  Bufs b{};
  b.whole_hist = sp.b[f].whole_hist;
  b.whole_sums = sp.b[f].whole_sums;
  b.lut8 = sp.b[f].lut8;
  b.q16 = sp.b[f].q16;
  b.weights = sp.b[f].weights;
  const SetFrames& fp = sp.f[f];
  const int s0 = uniform(g.wg_seg[w]), s1 = uniform(g.wg_seg[w + 1]);
  int prev = -1;
  for (int s = s0; s < s1;) {
    const int cam = uniform(g.tiles[s].cam);
    if (!cam_active(g, cam)) {
      ++s;
      continue;
    }
    s = apply_tile_dispatch<true, true, true, VBLEND>(g, fp, b, s, s1, L, cam != prev);
    __syncthreads();
    prev = cam;
  }
}

// start / stop (may be NULL): events that take the dispatch's own start and
// end times (no marker packets around it).
hipError_t launch_apply(const Geo& g, const FramePtrs& fp, const Bufs& b, bool write, bool stats, hipStream_t st,
                        hipEvent_t start, hipEvent_t stop) {
  const dim3 grid(g.n_wg), block(kThreads);
  if (g.vblend && write && stats)
    hipExtLaunchKernelGGL((k_apply<true, true, true>), grid, block, 0, st, start, stop, 0u, g, fp, b);
  else if (g.vblend && write)
    hipExtLaunchKernelGGL((k_apply<true, false, true>), grid, block, 0, st, start, stop, 0u, g, fp, b);
  else if (write && stats)
    hipExtLaunchKernelGGL((k_apply<true, true, false>), grid, block, 0, st, start, stop, 0u, g, fp, b);
  else if (write)
    hipExtLaunchKernelGGL((k_apply<true, false, false>), grid, block, 0, st, start, stop, 0u, g, fp, b);
  else if (stats)
    hipExtLaunchKernelGGL((k_apply<false, true, false>), grid, block, 0, st, start, stop, 0u, g, fp, b);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

const void* apply_kernel(const Geo& g, bool write, bool stats) {
  if (g.vblend && write && stats) return reinterpret_cast<const void*>(&k_apply<true, true, true>);
  if (g.vblend && write) return reinterpret_cast<const void*>(&k_apply<true, false, true>);
  if (write && stats) return reinterpret_cast<const void*>(&k_apply<true, true, false>);
  if (write) return reinterpret_cast<const void*>(&k_apply<true, false, false>);
  if (stats) return reinterpret_cast<const void*>(&k_apply<false, true, false>);
  return nullptr;
}

hipError_t launch_apply_sets(const Geo& g, const SetPtrs& sp, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if (sp.n_sets < 1 || sp.n_sets > kSetsMax || g.n_cams > kSetCams) return hipErrorInvalidValue;
  const dim3 grid(g.n_wg * sp.n_sets), block(kThreads);
  if (g.vblend) hipExtLaunchKernelGGL((k_apply_sets<true>), grid, block, 0, st, start, stop, 0u, g, sp);
  else hipExtLaunchKernelGGL((k_apply_sets<false>), grid, block, 0, st, start, stop, 0u, g, sp);
  return hipGetLastError();
}

}  // namespace rc
