// Estimate and table kernels of section 3.1: one thread per (camera, side,
// block, channel) for the affine fit, one workgroup per (camera, side, block)
// for the tables, one thread per column for the blend weights; the
// look-ahead frame-set kernel (the apply of one frame-set in the same launch
// as the seam estimate of the next).
#include "dev_apply.h"
#include "dev_estimate.h"
#include "dev_motion.h"
#include "dev_stats.h"
#include "rt_ahead_internal.h"

namespace rc {

__global__ __launch_bounds__(kThreads) void k_estimate(Geo g, Bufs b) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < g.n_cams * 2 * g.n_blocks * kCS && cam_active(g, u / (2 * g.n_blocks * kCS))) estimate_unit(g, b, u);
}

// The quantile fit of every unit (RT_FIT_QUANTILE), one wave per (camera,
// side, block, channel) unit: the wave gathers the quantiles of the unit's
// band and of the band it faces from the band histograms, its first lane fits
// and updates the state.
__global__ __launch_bounds__(kThreads) void k_estimate_quantile(Geo g, Bufs b) {
  __shared__ uint32_t cum[kThreads / kWave][2 * kNB];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int u = uniform((int32_t)(blockIdx.x * (kThreads / kWave) + wave));
  const int nb = g.n_blocks;
  if (u >= g.n_cams * 2 * nb * kCS) return;    // the whole wave
  const int c = u % kCS, j = (u / kCS) % nb, s = (u / (kCS * nb)) & 1, k = u / (kCS * nb * 2);
  if (!cam_active(g, k)) return;
  const DevCam cam = uniform_cam(g.cams[k]);
  const int fc = cam.face_cam[s];
  const int64_t uf = fc < 0 ? -1 : unit_index(fc, cam.face_side[s], j, c, nb);
  const uint64_t n_own = b.band_sums[(int64_t)u * 3];
  const uint64_t n_fac = uf < 0 ? 0 : b.band_sums[uf * 3];
  QSums q = {0, 0, 0, 0, 0};
  if (c < cam.channels && uf >= 0 && n_own != 0 && n_fac != 0)
    q = wave_quantile_sums(b.band_hist + (int64_t)u * kNB, b.band_hist + uf * kNB, cam.bit_depth - 8 > 0 ? cam.bit_depth - 8 : 0,
                           cum[wave], lane);
  if (lane == 0) {
    double a, bb;
    const int st = fit_quantile(g, cam.channels, c, uf >= 0, n_own, n_fac, q, true, a, bb);
    temporal_update(g, b.params, b.valid, u, st, a, bb);
  }
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

// Band statistics, estimate and tables of a frame-set in one launch, one
// workgroup per (camera k, block j): it takes the right band of camera k, the
// band that faces it (the left band of the next camera of the ring) and, at
// the start of an open ring, camera k's left band, which faces nothing.
// Every unit is taken exactly once, and a unit's estimate needs only its own
// band and the one it faces, so after the statistics of its bands the
// workgroup fits those units and builds their tables with no other
// workgroup involved.  WIDE: 2 x kThreads threads whose halves gather two
// bands at the same time (for rigs with few seam blocks, where the launch
// is latency-bound; beside the apply kernels of a pipeline the 256-thread
// form is faster, as its workgroups fit more easily on busy compute units).
// Same results as k_band_stats, k_estimate, k_build_lut and k_weights in
// sequence (the whole-frame statistics that the frame-set's apply pass
// accumulates are cleared here too, when given).  REMOVAL: the band passes
// also sum the pixels that do not move against the previous frames, and
// each unit takes the object-removal fit or the smoothing fallback
// (removal_step), as k_motion_stats and k_estimate_removal would.
template <bool WIDE, bool REMOVAL, bool QFIT, typename Lds>
__device__ __attribute__((always_inline)) void band_estimate_body(const Geo& g, const FramePtrs& fp,
                                                                  const PrevPtrs& pp, const Bufs& b,
                                                                  const Removal& rm, Lds* L, int bid, int nblk) {
  static_assert(!(REMOVAL && QFIT), "object removal keeps only the moments of the kept pixels");
  constexpr int NT = WIDE ? 2 * kThreads : kThreads;
  // This kernel's chain of dependent steps is what the next apply waits
  // for; its waves take issue priority over the apply waves they share
  // compute units with (measured on MI355X: 628 -> 674 GPix/s in the
  // pipelined frame-set loop).
  __builtin_amdgcn_s_setprio(3);
  __shared__ uint64_t sums[3][9];            // (n, S1, S2) per channel of the units taken
  __shared__ uint64_t kept[REMOVAL ? 3 : 1][9];   // the same over their kept pixels
  __shared__ double ab[3][kCS][2];           // their maps after the fit
  // QFIT: the quantile sums of the facing pair (u0, u1) per channel, wave c
  // taking channel c.
  __shared__ uint32_t qcum[QFIT ? kCS : 1][QFIT ? 2 * kNB : 1];
  __shared__ QSums qs[QFIT ? kCS : 1];
  const int nb = g.n_blocks;
  const int k = bid / nb, j = bid - (bid / nb) * nb;
  const int tid = threadIdx.x;
  // WIDE: each half is whole waves, so its unit (camera, frame pointer) is
  // uniform per wave and stays in scalar registers.
  const int half = WIDE ? uniform((int32_t)(tid / kThreads)) : 0, ltid = tid - half * kThreads;
  if (b.whole_hist) zero_whole(g, b, bid * NT + tid, nblk * NT);
  if (!cam_active(g, k)) return;
  const DevCam& cam = g.cams[k];
  // Units taken, n of them: u0 the right band of camera k; u1 the band it
  // faces, if any; then the left band of camera k if it faces nothing.
  // Only u0 and u1 face each other.
  const int fc = uniform(cam.face_cam[1]);
  const int u0 = (k * 2 + 1) * nb + j;
  const int uf = fc < 0 ? -1 : (fc * 2 + uniform(cam.face_side[1])) * nb + j;
  const int ul = uniform(cam.face_cam[0]) < 0 ? k * 2 * nb + j : -1;
  const int u1 = uf >= 0 ? uf : ul;
  const int u2 = uf >= 0 ? ul : -1;
  const int n = 1 + (u1 >= 0) + (u2 >= 0);
  auto unit_at = [&](int i) { return i == 0 ? u0 : (i == 1 ? u1 : u2); };
  auto band_pass = [&](int i, Lds& Li, int t) {
    if constexpr (REMOVAL) band_unit_motion_dispatch(g, fp, pp, b, rm, unit_at(i), Li, sums[i], kept[i], t);
    else band_unit_dispatch(g, fp, b, unit_at(i), Li, sums[i], t);
  };
  constexpr int kBarriers = REMOVAL ? kMotionBarriers : kBandBarriers;
  // Thread 64 t + c fits channel c of unit t: its state is read now, ahead
  // of the band passes.
  const int t = tid / kWave, c = tid % kWave;
  const bool fitter = t < n && c < kCS;
  const int64_t u = fitter ? (int64_t)unit_at(t) * kCS + c : 0;
  double p0 = 0.0, p1 = 0.0;
  uint8_t v = 0;
  if (fitter) {
    p0 = b.params[u * 2];
    p1 = b.params[u * 2 + 1];
    v = b.valid[u];
  }
  if (WIDE) {
    // Units 2p and 2p + 1 in pass p, one per half; a half without a unit
    // passes the same barriers.
    for (int p = 0; 2 * p < n; ++p) {
      if (p) __syncthreads();
      const int i = 2 * p + half;
      if (i < n) {
        band_pass(i, L[WIDE ? half : 0], ltid);
      } else {
        for (int w = 0; w < kBarriers; ++w) __syncthreads();
      }
    }
  } else {
    for (int i = 0; i < n; ++i) {
      if (i) __syncthreads();
      band_pass(i, L[0], tid);
    }
  }
  if (j == 0)
    for (int col = tid; col < g.w_max; col += NT)
      b.weights[(int64_t)k * g.w_max + col] = (uint16_t)blend_weight(cam.width, col);
  __syncthreads();
  if constexpr (QFIT) {
    // Only u0 and u1 face each other; the band histograms were written by
    // this workgroup's band passes.
    const int wv = uniform((int32_t)(tid / kWave));
    if (uf >= 0 && wv < uniform(cam.channels)) {
      const int shift = cam.bit_depth > 8 ? cam.bit_depth - 8 : 0;
      const QSums q = wave_quantile_sums(b.band_hist + ((int64_t)u0 * kCS + wv) * kNB,
                                         b.band_hist + ((int64_t)uf * kCS + wv) * kNB, shift, qcum[wv], tid % kWave);
      if (tid % kWave == 0) qs[wv] = q;
    }
    __syncthreads();
  }
  if (fitter) {
    const int other = (uf >= 0 && t < 2) ? 1 - t : -1;
    const uint64_t* fac = other >= 0 ? &sums[other][c * 3] : nullptr;
    const int channels = uniform(g.cams[unit_at(t) / (2 * nb)].channels);
    if constexpr (REMOVAL) {
      const uint64_t* kfac = other >= 0 ? &kept[other][c * 3] : nullptr;
      const int m = removal_method(&sums[t][0], other >= 0 ? &sums[other][0] : nullptr, &kept[t][0],
                                   other >= 0 ? &kept[other][0] : nullptr, rm.min_kept);
      removal_step(g, m, channels, c, &sums[t][c * 3], fac, &kept[t][c * 3], kfac, p0, p1, v);
      if (c == 0 && rm.method) rm.method[unit_at(t)] = (uint8_t)m;
    } else {
      double a, bb;
      int st;
      if (QFIT && fac)
        st = fit_quantile(g, channels, c, true, sums[t][c * 3], sums[other][c * 3], qs[QFIT ? c : 0], t == 0, a,
                          bb);
      else
        st = fit_sums(g, channels, c, &sums[t][c * 3], fac, a, bb);
      temporal_step(g, st, a, bb, p0, p1, v);
    }
    b.params[u * 2] = p0;
    b.params[u * 2 + 1] = p1;
    b.valid[u] = v;
    ab[t][c][0] = p0;
    ab[t][c][1] = p1;
  }
  __syncthreads();
  for (int w = half; w < n; w += (WIDE ? 2 : 1)) lut_entry_ab(g, b, unit_at(w), ltid, ab[w]);
}

template <bool WIDE, bool QFIT>
__global__ __launch_bounds__(WIDE ? 2 * kThreads : kThreads) void k_band_estimate(Geo g, FramePtrs fp, Bufs b) {
  __shared__ StatsLds L[WIDE ? 2 : 1];
  PrevPtrs pp;
  Removal rm;
  band_estimate_body<WIDE, false, QFIT>(g, fp, pp, b, rm, L, (int)blockIdx.x, (int)gridDim.x);
}

template <bool WIDE>
__global__ __launch_bounds__(WIDE ? 2 * kThreads : kThreads) void k_band_estimate_removal(Geo g, FramePtrs fp,
                                                                                          PrevPtrs pp, Bufs b,
                                                                                          Removal rm) {
  __shared__ MotionLds L[WIDE ? 2 : 1];
  band_estimate_body<WIDE, true, false>(g, fp, pp, b, rm, L, (int)blockIdx.x, (int)gridDim.x);
}

// Band statistics with the kept sums, one workgroup per (camera, side, block).
__global__ __launch_bounds__(kThreads) void k_motion_stats(Geo g, FramePtrs fp, PrevPtrs pp, Bufs b, Removal rm) {
  __shared__ MotionLds L;
  band_unit_motion_dispatch(g, fp, pp, b, rm, blockIdx.x, L, nullptr, nullptr, threadIdx.x);
}

// Removal fit or fallback of every (camera, side, block, channel) unit from
// the band and kept sums in the caller's layout; the channel-0 thread of a
// unit writes its method.
__global__ __launch_bounds__(kThreads) void k_estimate_removal(Geo g, Bufs b, Removal rm) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= g.n_cams * 2 * g.n_blocks * kCS) return;
  const int nb = g.n_blocks;
  const int c = u % kCS, j = (u / kCS) % nb, s = (u / (kCS * nb)) & 1, k = u / (kCS * nb * 2);
  if (!cam_active(g, k)) return;
  const DevCam& cam = g.cams[k];
  const int fc = cam.face_cam[s];
  const int64_t uo = unit_index(k, s, j, 0, nb);
  const int64_t uf = fc < 0 ? -1 : unit_index(fc, cam.face_side[s], j, 0, nb);
  const uint64_t* own = b.band_sums + uo * 3;
  const uint64_t* kown = rm.kept_sums + uo * 3;
  const uint64_t* fac = uf < 0 ? nullptr : b.band_sums + uf * 3;
  const uint64_t* kfac = uf < 0 ? nullptr : rm.kept_sums + uf * 3;
  const int m = removal_method(own, fac, kown, kfac, rm.min_kept);
  double p0 = b.params[(int64_t)u * 2], p1 = b.params[(int64_t)u * 2 + 1];
  uint8_t v = b.valid[u];
  removal_step(g, m, cam.channels, c, own + c * 3, fac ? fac + c * 3 : nullptr, kown + c * 3,
               kfac ? kfac + c * 3 : nullptr, p0, p1, v);
  b.params[(int64_t)u * 2] = p0;
  b.params[(int64_t)u * 2 + 1] = p1;
  b.valid[u] = v;
  if (c == 0 && rm.method) rm.method[u / kCS] = (uint8_t)m;
}

// A frame-set of the look-ahead loop in one launch: workgroups [0, n_est)
// take the seam blocks of frame-set t + 1 (fe, be: its band statistics,
// estimate and tables, and the clearing of its whole-frame statistics, as
// k_band_estimate), the others apply frame-set t (fa, ba: with the tables an
// earlier launch built, as k_apply with statistics).  The two parts share no
// buffer and neither waits for the other; consecutive launches on a stream
// chain the estimates in order.
union AheadLds {
  ApplyLds a;
  StatsLds s;
};
template <bool VBLEND, bool QFIT>
__global__ __launch_bounds__(kThreads) void k_frameset_ahead(Geo g, FramePtrs fa, Bufs ba, FramePtrs fe, Bufs be,
                                                             int n_est) {
  __shared__ AheadLds U;
  const int bid = (int)blockIdx.x;
  if (bid < n_est) {
    PrevPtrs pp;
    Removal rm;
    band_estimate_body<false, false, QFIT>(g, fe, pp, be, rm, &U.s, bid, n_est);
    return;
  }
  const int w = bid - n_est;
  const int s0 = uniform(g.wg_seg[w]), s1 = uniform(g.wg_seg[w + 1]);
  int prev = -1;
  for (int s = s0; s < s1;) {
    const int cam = uniform(g.tiles[s].cam);
    if (!cam_active(g, cam)) {
      ++s;
      continue;
    }
    s = apply_tile_dispatch<true, true, true, VBLEND>(g, fa, ba, s, s1, U.a, cam != prev);
    __syncthreads();
    prev = cam;
  }
}

hipError_t launch_frameset_ahead(const Geo& g, const FramePtrs* fa, const Bufs& ba, const FramePtrs* fe,
                                 const Bufs& be, hipStream_t st) {
  const int n_est = fe ? g.n_cams * g.n_blocks : 0, n_app = fa ? g.n_wg : 0;
  if (n_est + n_app == 0) return hipSuccess;
  const FramePtrs none = {};
  const FramePtrs& a = fa ? *fa : none;
  const FramePtrs& e = fe ? *fe : none;
  const dim3 grid(n_est + n_app), block(kThreads);
  const bool q = g.fit == RT_FIT_QUANTILE;
  if (g.vblend && q) hipLaunchKernelGGL((k_frameset_ahead<true, true>), grid, block, 0, st, g, a, ba, e, be, n_est);
  else if (g.vblend) hipLaunchKernelGGL((k_frameset_ahead<true, false>), grid, block, 0, st, g, a, ba, e, be, n_est);
  else if (q) hipLaunchKernelGGL((k_frameset_ahead<false, true>), grid, block, 0, st, g, a, ba, e, be, n_est);
  else hipLaunchKernelGGL((k_frameset_ahead<false, false>), grid, block, 0, st, g, a, ba, e, be, n_est);
  return hipGetLastError();
}

// Seam blocks up to which the wide form is launched.
constexpr int kWideSeamBlocks = 64;

hipError_t launch_band_estimate(const Geo& g, const FramePtrs& fp, const Bufs& b, hipStream_t st) {
  const int blocks = g.n_cams * g.n_blocks;
  const bool wide = blocks <= kWideSeamBlocks, q = g.fit == RT_FIT_QUANTILE;
  const dim3 grid(blocks), block(wide ? 2 * kThreads : kThreads);
  if (wide && q) hipLaunchKernelGGL((k_band_estimate<true, true>), grid, block, 0, st, g, fp, b);
  else if (wide) hipLaunchKernelGGL((k_band_estimate<true, false>), grid, block, 0, st, g, fp, b);
  else if (q) hipLaunchKernelGGL((k_band_estimate<false, true>), grid, block, 0, st, g, fp, b);
  else hipLaunchKernelGGL((k_band_estimate<false, false>), grid, block, 0, st, g, fp, b);
  return hipGetLastError();
}

const void* band_estimate_kernel(const Geo& g) {
  const bool wide = g.n_cams * g.n_blocks <= kWideSeamBlocks, q = g.fit == RT_FIT_QUANTILE;
  if (wide && q) return reinterpret_cast<const void*>(&k_band_estimate<true, true>);
  if (wide) return reinterpret_cast<const void*>(&k_band_estimate<true, false>);
  if (q) return reinterpret_cast<const void*>(&k_band_estimate<false, true>);
  return reinterpret_cast<const void*>(&k_band_estimate<false, false>);
}

hipError_t launch_band_estimate_removal(const Geo& g, const FramePtrs& fp, const PrevPtrs& pp, const Bufs& b,
                                        const Removal& rm, hipStream_t st) {
  const int blocks = g.n_cams * g.n_blocks;
  if (blocks <= kWideSeamBlocks)
    hipLaunchKernelGGL(k_band_estimate_removal<true>, dim3(blocks), dim3(2 * kThreads), 0, st, g, fp, pp, b, rm);
  else
    hipLaunchKernelGGL(k_band_estimate_removal<false>, dim3(blocks), dim3(kThreads), 0, st, g, fp, pp, b, rm);
  return hipGetLastError();
}

hipError_t launch_motion_stats(const Geo& g, const FramePtrs& fp, const PrevPtrs& pp, const Bufs& b,
                               const Removal& rm, hipStream_t st) {
  hipLaunchKernelGGL(k_motion_stats, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, fp, pp, b, rm);
  return hipGetLastError();
}

hipError_t launch_estimate_removal(const Geo& g, const Bufs& b, const Removal& rm, hipStream_t st) {
  const int total = g.n_cams * 2 * g.n_blocks * kCS;
  hipLaunchKernelGGL(k_estimate_removal, dim3((total + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, b, rm);
  return hipGetLastError();
}

hipError_t launch_estimate(const Geo& g, const Bufs& b, hipStream_t st) {
  const int total = g.n_cams * 2 * g.n_blocks * kCS;
  if (g.fit == RT_FIT_QUANTILE) {
    constexpr int per = kThreads / kWave;
    hipLaunchKernelGGL(k_estimate_quantile, dim3((total + per - 1) / per), dim3(kThreads), 0, st, g, b);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_estimate, dim3((total + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, b);
  return hipGetLastError();
}

hipError_t launch_weights(const Geo& g, const Bufs& b, hipStream_t st) {
  const int64_t n = (int64_t)g.n_cams * g.w_max;
  hipLaunchKernelGGL(k_weights, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, g, b);
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
