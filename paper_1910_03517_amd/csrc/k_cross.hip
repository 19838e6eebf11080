// Cross-channel 3x3 maps (section 5 proposes linear maps across the colour
// channels instead of one affine map per channel): the cross sums of every
// band, the fit of M and t per (camera, side, block), their Q16 form, and the
// apply pass, for rigs of 8-bit RGB cameras.
//
// Fit of one side: mu and the covariance C from the exact sums (binary64),
// the Cholesky factors L_own, L_fac of both bands, the shared factor
// L* = (L_own + L_fac) / 2 and mean mu* = (mu_own + mu_fac) / 2, then
// M = L* L_own^-1 (M L_own = L* solved row by row from the last column) and
// t = mu* - M mu_own.  Every step is one binary64 operation in the written
// order, contraction off.  When either covariance has a pivot <= 0, or M has
// a diagonal entry outside [a_min, a_max] or an off-diagonal entry beyond
// a_max in magnitude, the side takes the per-channel fits of the plain
// estimate instead (a diagonal M).
#include "dev_apply.h"

#pragma clang fp contract(off)

namespace rc {

constexpr int kX3 = 12;   // parameters of one map
constexpr int kXU = 4;    // rows in flight per thread in the apply

// ----------------------------------------------------------------- statistics

// Cross sums of the band of unit (k, s, j) = blockIdx.x, one workgroup each.
__global__ __launch_bounds__(kThreads) void k_cross_stats(Geo g, FramePtrs fp, CrossBufs x) {
  __shared__ unsigned long long red[3 * 16];
  const int nb = g.n_blocks, unit = blockIdx.x;
  const int k = unit / (2 * nb), s = (unit / nb) & 1, j = unit % nb;
  if (!cam_active(g, k)) return;
  const DevCam cam = uniform_cam(g.cams[k]);
  const int r0 = (int)((int64_t)j * cam.height / nb), r1 = (int)((int64_t)(j + 1) * cam.height / nb);
  const int band = cam.band, c0 = s == 0 ? 0 : cam.width - band;
  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[k], cam);
  const int pitch = (int)cam.pitch;
  unsigned long long p01 = 0, p02 = 0, p12 = 0;
  const int total = (r1 - r0) * band;
  for (int i = threadIdx.x; i < total; i += kThreads) {
    const int row = r0 + i / band, col = c0 + i % band;
    const int off = row * pitch + col * 3;
    const uint32_t x0 = __builtin_amdgcn_raw_buffer_load_b8(rin, off, 0, 0);
    const uint32_t x1 = __builtin_amdgcn_raw_buffer_load_b8(rin, off + 1, 0, 0);
    const uint32_t x2 = __builtin_amdgcn_raw_buffer_load_b8(rin, off + 2, 0, 0);
    p01 += x0 * x1;
    p02 += x0 * x2;
    p12 += x1 * x2;
  }
  block_sums(
      3, [&](int i) -> unsigned long long { return i == 0 ? p01 : (i == 1 ? p02 : p12); },
      [&](int i, unsigned long long tot) { x.cross[(int64_t)unit * 3 + i] = tot; }, red);
}

// ----------------------------------------------------------------- estimate

struct MeanCov {
  double mu[3];
  double cov[3][3];
};

// sums: (n, S1, S2) of channels 0..2; cross: (S_RG, S_RB, S_GB).
__device__ inline MeanCov mean_cov(const uint64_t* sums, const uint64_t* cross) {
  MeanCov m;
  const double n = (double)sums[0];
  for (int c = 0; c < 3; ++c) m.mu[c] = (double)sums[c * 3 + 1] / n;
  for (int c = 0; c < 3; ++c) {
    const double ex = (double)sums[c * 3 + 2] / n;
    const double m2 = m.mu[c] * m.mu[c];
    const double v = ex - m2;
    m.cov[c][c] = v > 0.0 ? v : 0.0;
  }
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int i = 0; i < 3; ++i) {
    const double ex = (double)cross[i] / n;
    const double m2 = m.mu[pa[i]] * m.mu[pb[i]];
    m.cov[pa[i]][pb[i]] = m.cov[pb[i]][pa[i]] = ex - m2;
  }
  return m;
}

// Lower Cholesky factor of C; false when a pivot is not positive.
__device__ inline bool cholesky3(const double (&C)[3][3], double (&L)[3][3]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) L[r][c] = 0.0;
  if (!(C[0][0] > 0.0)) return false;
  L[0][0] = __builtin_sqrt(C[0][0]);
  L[1][0] = C[1][0] / L[0][0];
  L[2][0] = C[2][0] / L[0][0];
  const double p11 = C[1][1] - L[1][0] * L[1][0];
  if (!(p11 > 0.0)) return false;
  L[1][1] = __builtin_sqrt(p11);
  L[2][1] = (C[2][1] - L[2][0] * L[1][0]) / L[1][1];
  const double p22 = (C[2][2] - L[2][0] * L[2][0]) - L[2][1] * L[2][1];
  if (!(p22 > 0.0)) return false;
  L[2][2] = __builtin_sqrt(p22);
  return true;
}

// (M, t) of the own side into m[12]; false when a band is empty.
__device__ inline bool fit_cross(const Geo& g, const uint64_t* os, const uint64_t* ox, const uint64_t* fs,
                                 const uint64_t* fx, double (&m)[kX3]) {
  if (os[0] == 0 || fs[0] == 0) return false;
  const MeanCov mo = mean_cov(os, ox), mf = mean_cov(fs, fx);
  double Lo[3][3], Lf[3][3], M[3][3];
  bool ok = cholesky3(mo.cov, Lo);
  ok = cholesky3(mf.cov, Lf) && ok;
  if (ok) {
    for (int r = 0; r < 3; ++r) {
      double ls[3];
      for (int c = 0; c < 3; ++c) ls[c] = (Lo[r][c] + Lf[r][c]) / 2.0;
      const double m2 = ls[2] / Lo[2][2];
      const double m1 = (ls[1] - m2 * Lo[2][1]) / Lo[1][1];
      const double m0 = ((ls[0] - m1 * Lo[1][0]) - m2 * Lo[2][0]) / Lo[0][0];
      M[r][0] = m0;
      M[r][1] = m1;
      M[r][2] = m2;
    }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const double v = M[r][c];
        const bool good = r == c ? (v >= g.a_min && v <= g.a_max) : (v >= -g.a_max && v <= g.a_max);
        ok = ok && good;
      }
  }
  if (!ok) {
    for (int i = 0; i < kX3; ++i) m[i] = 0.0;
    for (int c = 0; c < 3; ++c) {
      double a, bb;
      (void)fit_sums(g, 3, c, os + c * 3, fs + c * 3, a, bb);
      m[c * 4] = a;
      m[9 + c] = bb;
    }
    return true;
  }
  for (int r = 0; r < 3; ++r) {
    const double mus = (mo.mu[r] + mf.mu[r]) / 2.0;
    const double mx = (M[r][0] * mo.mu[0] + M[r][1] * mo.mu[1]) + M[r][2] * mo.mu[2];
    for (int c = 0; c < 3; ++c) m[r * 3 + c] = M[r][c];
    m[9 + r] = mus - mx;
  }
  return true;
}

// One thread per (camera, side, block): fit, then the temporal step.
__global__ __launch_bounds__(kThreads) void k_estimate_cross(Geo g, Bufs b, CrossBufs x) {
  const int nb = g.n_blocks;
  const int u = blockIdx.x * kThreads + threadIdx.x;
  if (u >= g.n_cams * 2 * nb) return;
  const int k = u / (2 * nb), s = (u / nb) & 1, j = u % nb;
  if (!cam_active(g, k)) return;
  const DevCam& cam = g.cams[k];
  double* p = x.params3 + (int64_t)u * kX3;
  const bool had = x.valid3[u] != 0;
  double m[kX3];
  const int fc = cam.face_cam[s];
  const int64_t uf = fc < 0 ? -1 : ((int64_t)fc * 2 + cam.face_side[s]) * nb + j;
  const bool fresh = uf >= 0 && fit_cross(g, b.band_sums + (int64_t)u * kCS * 3, x.cross + (int64_t)u * 3,
                                          b.band_sums + uf * kCS * 3, x.cross + uf * 3, m);
  if (!fresh) {
    if (uf >= 0 && had) return;                 // no estimate: keep the state
    for (int i = 0; i < kX3; ++i) p[i] = (i < 9 && i % 4 == 0) ? 1.0 : 0.0;
    x.valid3[u] = uf < 0 ? 1 : 0;               // identity without a facing band
    return;
  }
  if (g.mode == RT_MODE_SMOOTHING && had) {
    const double keep = 1.0 - g.alpha;
    for (int i = 0; i < kX3; ++i) {
      const double tp = keep * p[i];
      const double tn = g.alpha * m[i];
      m[i] = tp + tn;
    }
  }
  for (int i = 0; i < kX3; ++i) p[i] = m[i];
  x.valid3[u] = 1;
}

// q3 = round_half_even(params3 * 65536), one thread per parameter.
__global__ __launch_bounds__(kThreads) void k_build_cross(Geo g, CrossBufs x) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)g.n_cams * 2 * g.n_blocks * kX3) return;
  if (!cam_active(g, (int)(i / ((int64_t)2 * g.n_blocks * kX3)))) return;
  x.q3[i] = (int64_t)__builtin_rint(x.params3[i] * 65536.0);
}

// ----------------------------------------------------------------- apply

// Whether every row r of both sides' maps can be evaluated in 32-bit
// integers: |A| < 2^23 (24-bit multiplies) and A_r . x + B_r + 2^15 inside
// int32 for every x in [0, 255]^3.
__device__ inline bool cross_small(const int64_t (&q)[2][kX3]) {
  bool ok = true;
#pragma unroll
  for (int sd = 0; sd < 2; ++sd)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      int64_t lo = q[sd][9 + r] + 32768, hi = lo;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t a = q[sd][r * 3 + c];
        ok = ok && a < (1 << 23) && a > -(1 << 23);
        lo += a < 0 ? 255 * a : 0;
        hi += a > 0 ? 255 * a : 0;
      }
      ok = ok && lo >= INT32_MIN && hi <= INT32_MAX;
    }
  return ok;
}

// The blended sample of channel r: f = clamp((A_r . x + B_r + 2^15) >> 16,
// 0, 255), y = ((256 - w) x_r + w f + 128) >> 8.
// y = ((256 - w) x + w f + 128) >> 8 as one dot product of (x, f) with (256 - w, w).
__device__ inline uint32_t cross_blend(uint32_t x, uint32_t f, uint32_t wp) {
  return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, x | (f << 16)), __builtin_bit_cast(u16x2, wp), 128u,
                                false) >> 8;
}

// One row of a 4-pixel group with a 32-bit map a (B + 2^15 last) shared by
// its four pixels: the histogram of its samples (STATS), then per sample the
// map clamped in place, clamp(v, 0, 2^24 - 1) & 0xffff0000 = f << 16 for the
// arithmetic v >> 16 (so f lands in the high half next to x), the blend as
// one dot product, and the four results of a dword gathered by byte permutes.
template <bool STATS>
__device__ inline void cross_group_fast(const uint32_t (&d)[3], uint32_t (&o)[3], int npx, const uint32_t (&wp)[4],
                                        ApplyLds& L, int hrep, const int32_t (&a)[kX3]) {
  uint32_t raw[12];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    uint32_t xs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int i = p * 3 + c;
      xs[c] = (d[i >> 2] >> (8 * (i & 3))) & 0xffu;
      if (STATS && p < npx)
        __hip_atomic_fetch_add(&L.hist[hist_word(c, xs[c]) * kRep + hrep], 1u << hist_shift(xs[c]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      int32_t v = a[r * 3] * (int32_t)xs[0] + a[r * 3 + 1] * (int32_t)xs[1] + a[r * 3 + 2] * (int32_t)xs[2] + a[9 + r];
      v = v < 0 ? 0 : (v > 0xffffff ? 0xffffff : v);
      const uint32_t xf = ((uint32_t)v & 0xffff0000u) | xs[r];
      raw[p * 3 + r] = p < npx ? __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, xf),
                                                        __builtin_bit_cast(u16x2, wp[p]), 128u, false)
                               : 0u;
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) o[q] = pack_raw4(raw[4 * q], raw[4 * q + 1], raw[4 * q + 2], raw[4 * q + 3]);
}

// Segment ti with the cross-channel maps of its block; optional whole-frame
// statistics as in the plain apply (first clears, last flushes).  SMALL (the
// maps fit 32-bit arithmetic, cross_small): the groups of four pixels that
// lie on one side take that side's map, the same for every lane (so it stays
// in scalar registers), with kXU rows of loads in flight.  The group holding
// the image centre, and every group when the maps need 64-bit arithmetic, go
// sample by sample with the map read from LDS.
template <bool STATS, bool SMALL>
__device__ __attribute__((always_inline)) void cross_tile(const Geo& g, const FramePtrs& fp, const Bufs& b,
                                                          const CrossBufs& x, int ti, ApplyLds& L, bool first,
                                                          bool last, const int64_t (&q)[2][kX3]) {
  const int tid = threadIdx.x;
  const Tile t = uniform_tile(g.tiles[ti]);
  const DevCam cam = uniform_cam(g.cams[t.cam]);
  const int W = cam.width, half = cam.half, pitch = (int)cam.pitch;
  int64_t* qs = reinterpret_cast<int64_t*>(L.lut);   // [side][12]
  if (tid < 2 * kX3) qs[tid] = x.q3[(((int64_t)t.cam * 2 + tid / kX3) * g.n_blocks + t.block) * kX3 + tid % kX3];
  if (STATS && first)
    for (int i = tid; i < kHistWords; i += kThreads) L.hist[i] = 0;
  __syncthreads();
  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[t.cam], cam);
  const __amdgpu_buffer_rsrc_t rout = frame_rsrc(fp.out[t.cam], cam);
  const uint16_t* wrow = x.weights + (int64_t)t.cam * g.w_max;
  const int hrep = tid & (kRep - 1);
  const int ngroups = (W + 3) >> 2;
  // Both sides' maps in 32-bit form (uniform).
  int32_t aL[kX3], aR[kX3];
#pragma unroll
  for (int i = 0; i < kX3; ++i) {
    aL[i] = i >= 9 ? (int32_t)(q[0][i] + 32768) : (int32_t)((uint32_t)q[0][i] << 8) >> 8;
    aR[i] = i >= 9 ? (int32_t)(q[1][i] + 32768) : (int32_t)((uint32_t)q[1][i] << 8) >> 8;
  }
  // Group grp (four pixels) of every row of the segment: mode 0 / 1 all on
  // the left / right side with that side's map, 2 sample by sample.
  auto do_group = [&](int grp, int mode) {
    const int col0 = grp * 4, npx = min(4, W - col0);
    uint32_t wp[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint32_t w = p < npx ? (uint32_t)wrow[col0 + p] : 0u;
      wp[p] = (256u - w) | (w << 16);
    }
    auto rows_one_side = [&](const int32_t (&a)[kX3]) {
      for (int row = t.r0; row < t.r1; row += kXU) {
        uint32_t d[kXU][3];
#pragma unroll
        for (int u = 0; u < kXU; ++u) {
          const int off = (row + u) * pitch + col0 * 3;
          if (row + u < t.r1) {
            if (npx == 4) {
              load_group<3>(rin, off, d[u]);
            } else {
              d[u][0] = d[u][1] = d[u][2] = 0u;
#pragma unroll
              for (int i = 0; i < 12; ++i)
                if (i < 3 * npx)
                  d[u][i >> 2] |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rin, off + i, 0, 0) << (8 * (i & 3));
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kXU; ++u) {
          if (row + u < t.r1) {
            const int off = (row + u) * pitch + col0 * 3;
            uint32_t o[3];
            cross_group_fast<STATS>(d[u], o, npx, wp, L, hrep, a);
            if (npx == 4) {
              store_group<3>(rout, off, o);
            } else {
#pragma unroll
              for (int i = 0; i < 12; ++i)
                if (i < 3 * npx)
                  __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(o[i >> 2] >> (8 * (i & 3))), rout, off + i, 0, 0);
            }
          }
        }
      }
    };
    if (SMALL && mode == 0) {
      rows_one_side(aL);
    } else if (SMALL && mode == 1) {
      rows_one_side(aR);
    } else {
      // Sample by sample in 64-bit integers (exact for every map).
      for (int row = t.r0; row < t.r1; ++row) {
        const int off = row * pitch + col0 * 3;
#pragma unroll 1
        for (int p = 0; p < npx; ++p) {
          const uint32_t x0 = __builtin_amdgcn_raw_buffer_load_b8(rin, off + 3 * p, 0, 0);
          const uint32_t x1 = __builtin_amdgcn_raw_buffer_load_b8(rin, off + 3 * p + 1, 0, 0);
          const uint32_t x2 = __builtin_amdgcn_raw_buffer_load_b8(rin, off + 3 * p + 2, 0, 0);
          if (STATS) {
            __hip_atomic_fetch_add(&L.hist[hist_word(0, x0) * kRep + hrep], 1u << hist_shift(x0), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&L.hist[hist_word(1, x1) * kRep + hrep], 1u << hist_shift(x1), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&L.hist[hist_word(2, x2) * kRep + hrep], 1u << hist_shift(x2), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
          }
          const int base = col0 + p >= half ? kX3 : 0;
          const uint32_t w = (uint32_t)wrow[col0 + p], wpp = (256u - w) | (w << 16);
#pragma unroll 1
          for (int c = 0; c < 3; ++c) {
            int64_t v = qs[base + c * 3] * (int64_t)x0 + qs[base + c * 3 + 1] * (int64_t)x1 +
                        qs[base + c * 3 + 2] * (int64_t)x2 + qs[base + 9 + c] + 32768;
            v >>= 16;
            const uint32_t f = (uint32_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
            const uint32_t xc = c == 0 ? x0 : (c == 1 ? x1 : x2);
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)cross_blend(xc, f, wpp), rout, off + 3 * p + c, 0, 0);
          }
        }
      }
    }
  };
  if (SMALL) {
    // Threads take the all-left groups, then the all-right ones, so that
    // every wave but the last of each run follows one side's path; the group
    // holding the image centre (when half % 4 != 0) goes sample by sample.
    const int gL = half >> 2, gR = (half + 3) >> 2;
    for (int i = tid; i < gL; i += kThreads) do_group(i, 0);
    for (int i = tid; i < ngroups - gR; i += kThreads) do_group(gR + i, 1);
    if (gR > gL && tid == 0) do_group(gL, 2);
  } else {
    for (int grp = tid; grp < ngroups; grp += kThreads) do_group(grp, 2);
  }
  if (STATS && (last || kPack)) flush_whole<3, 1>(g, b, t.cam, L, 0ull, 0ull);
}

template <bool STATS>
__global__ __launch_bounds__(kThreads) void k_apply_cross(Geo g, FramePtrs fp, Bufs b, CrossBufs x) {
  __shared__ ApplyLds L;
  const int s0 = uniform(g.wg_seg[blockIdx.x]), s1 = uniform(g.wg_seg[blockIdx.x + 1]);
  int prev = -1;
  for (int s = s0; s < s1; ++s) {
    const int cam = uniform(g.tiles[s].cam);
    if (!cam_active(g, cam)) continue;
    const bool last = s + 1 == s1 || uniform(g.tiles[s + 1].cam) != cam;
    const int blk = uniform(g.tiles[s].block);
    int64_t q[2][kX3];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int i = 0; i < kX3; ++i) q[sd][i] = uniform(x.q3[(((int64_t)cam * 2 + sd) * g.n_blocks + blk) * kX3 + i]);
    if (cross_small(q)) cross_tile<STATS, true>(g, fp, b, x, s, L, cam != prev, last, q);
    else cross_tile<STATS, false>(g, fp, b, x, s, L, cam != prev, last, q);
    __syncthreads();
    prev = cam;
  }
}

// ----------------------------------------------------------------- launchers

hipError_t launch_cross_stats(const Geo& g, const FramePtrs& fp, const CrossBufs& x, hipStream_t st) {
  hipLaunchKernelGGL(k_cross_stats, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, fp, x);
  return hipGetLastError();
}

hipError_t launch_estimate_cross(const Geo& g, const Bufs& b, const CrossBufs& x, hipStream_t st) {
  const int n = g.n_cams * 2 * g.n_blocks;
  hipLaunchKernelGGL(k_estimate_cross, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, b, x);
  return hipGetLastError();
}

hipError_t launch_build_cross(const Geo& g, const CrossBufs& x, hipStream_t st) {
  const int64_t n = (int64_t)g.n_cams * 2 * g.n_blocks * kX3;
  hipLaunchKernelGGL(k_build_cross, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, g, x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  Bufs b{};
  b.weights = x.weights;
  return launch_weights(g, b, st);
}

hipError_t launch_apply_cross(const Geo& g, const FramePtrs& fp, const Bufs& b, const CrossBufs& x, bool stats,
                              hipStream_t st) {
  if (stats) hipLaunchKernelGGL(k_apply_cross<true>, dim3(g.n_wg), dim3(kThreads), 0, st, g, fp, b, x);
  else hipLaunchKernelGGL(k_apply_cross<false>, dim3(g.n_wg), dim3(kThreads), 0, st, g, fp, b, x);
  return hipGetLastError();
}

}  // namespace rc
