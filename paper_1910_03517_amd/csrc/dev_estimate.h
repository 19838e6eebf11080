// Estimate and tables of section 3.1 as device functions: shared spectrum and
// per-channel affine fit of one unit with exponential smoothing, the
// fixed-point tables of one (camera, side, block), and the Q8 blend weights.
// Binary64 with contraction off: each result is the correctly rounded value
// of the expression as written.
#pragma once

#include "dev_common.h"

#pragma clang fp contract(off)

namespace rc {

struct Moments {
  double mu, var, sd;
};

__device__ inline Moments moments_of(uint64_t n, uint64_t s1, uint64_t s2) {
  Moments m;
  const double nf = (double)n;
  m.mu = (double)s1 / nf;
  const double ex2 = (double)s2 / nf;
  const double mu2 = m.mu * m.mu;
  double var = ex2 - mu2;
  if (var < 0.0) var = 0.0;
  m.var = var;
  m.sd = __builtin_sqrt(var);
  return m;
}

// Status of a (camera, side, block, channel) unit after the fit.
enum { kStNone = 0, kStNew = 1, kStIdentity = 2, kStUnused = 3 };

// The plain estimate of channel c of a unit of a camera with `channels`
// channels from the (n, S1, S2) of its own band and of the band it faces
// (fac NULL: no facing band), before any temporal step: kStNew with (a, b),
// kStNone (an empty band: keep the state), kStIdentity (no facing band),
// kStUnused (channel beyond the camera's).  Both sides of a seam derive the
// same shared moments because binary64 addition is commutative.
__device__ inline int fit_sums(const Geo& g, int channels, int c, const uint64_t* own, const uint64_t* fac, double& a,
                               double& bb) {
  a = 1.0;
  bb = 0.0;
  if (c >= channels) return kStUnused;
  if (!fac) return kStIdentity;
  if (own[0] == 0 || fac[0] == 0) return kStNone;
  const Moments mo = moments_of(own[0], own[1], own[2]);
  const Moments mf = moments_of(fac[0], fac[1], fac[2]);
  const double mu_s = (mo.mu + mf.mu) / 2.0;
  const double sd_s = (mo.sd + mf.sd) / 2.0;
  double aa = (mo.var == 0.0) ? 1.0 : sd_s / mo.sd;
  aa = aa < g.a_min ? g.a_min : aa;
  aa = aa > g.a_max ? g.a_max : aa;
  const double am = aa * mo.mu;
  a = aa;
  bb = mu_s - am;
  return kStNew;
}

// Quantile least-squares fit (RT_FIT_QUANTILE): the line through the pairs
// (x_i, (x_i + f_i) / 2) of the own and facing band's level-i quantiles,
// i = 0..63, with the bin centres doubled so that every sum is an exact
// integer.  One wave takes a facing pair's channel, lane i the level i.
constexpr int kQLevels = kWave;

struct QSums {
  int64_t sx, sf, sxx, sff, sxf;   // sums of 2x, 2f, (2x)^2, (2f)^2, (2x)(2f)
};

// Inclusive prefix sums of a 256-bin histogram (global memory) into cum (LDS),
// lane l taking bins 4l .. 4l + 3.
__device__ inline void wave_cum(const uint32_t* h, uint32_t* cum, int lane) {
  const uint32_t c0 = h[4 * lane], c1 = c0 + h[4 * lane + 1], c2 = c1 + h[4 * lane + 2], c3 = c2 + h[4 * lane + 3];
  uint32_t incl = c3;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += t;
  }
  const uint32_t base = incl - c3;
  cum[4 * lane] = base + c0;
  cum[4 * lane + 1] = base + c1;
  cum[4 * lane + 2] = base + c2;
  cum[4 * lane + 3] = base + c3;
}

// Smallest bin v with 2 M cum(v) >= (2 level + 1) n (binary search).
__device__ inline int quantile_bin(const uint32_t* cum, int level) {
  const uint64_t n = cum[kNB - 1];
  const uint64_t need = (uint64_t)(2 * level + 1) * n;
  int lo = 0, hi = kNB - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((uint64_t)(2 * kQLevels) * cum[mid] >= need) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Twice the centre of bin v in sample units: bins of 2^shift samples.
__device__ inline int64_t bin_centre2(int v, int shift) {
  return ((int64_t)(2 * v) << shift) + (1 << shift) - 1;
}

// The quantile sums of one channel of a facing pair (own histogram ho, facing
// hf, 256 bins each in global memory) by one whole wave; cum is 2 x 256 words
// of LDS owned by the wave.  Every lane returns the totals.
__device__ inline QSums wave_quantile_sums(const uint32_t* ho, const uint32_t* hf, int shift, uint32_t* cum,
                                           int lane) {
  wave_cum(ho, cum, lane);
  wave_cum(hf, cum + kNB, lane);
  // Lanes read what other lanes of the wave wrote.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int64_t x = bin_centre2(quantile_bin(cum, lane), shift);
  const int64_t f = bin_centre2(quantile_bin(cum + kNB, lane), shift);
  QSums q;
  q.sx = (int64_t)wave_sum_u64((unsigned long long)x);
  q.sf = (int64_t)wave_sum_u64((unsigned long long)f);
  q.sxx = (int64_t)wave_sum_u64((unsigned long long)(x * x));
  q.sff = (int64_t)wave_sum_u64((unsigned long long)(f * f));
  q.sxf = (int64_t)wave_sum_u64((unsigned long long)(x * f));
  __builtin_amdgcn_wave_barrier();
  return q;
}

// The quantile fit of channel c of a unit, own band = x of the sums when
// own_x, else f; n_own / n_fac are the bands' sample counts; has_fac false:
// no facing band.  Statuses as fit_sums.
__device__ inline int fit_quantile(const Geo& g, int channels, int c, bool has_fac, uint64_t n_own, uint64_t n_fac,
                                   const QSums& q, bool own_x, double& a, double& bb) {
  a = 1.0;
  bb = 0.0;
  if (c >= channels) return kStUnused;
  if (!has_fac) return kStIdentity;
  if (n_own == 0 || n_fac == 0) return kStNone;
  const int64_t M = kQLevels;
  const int64_t sx = own_x ? q.sx : q.sf, sf = own_x ? q.sf : q.sx;
  const int64_t sxx = own_x ? q.sxx : q.sff;
  const int64_t num = M * (sxx + q.sxf) - sx * (sx + sf);
  const int64_t den = M * sxx - sx * sx;
  double aa = den == 0 ? 1.0 : (double)num / (2.0 * (double)den);
  aa = aa < g.a_min ? g.a_min : aa;
  aa = aa > g.a_max ? g.a_max : aa;
  const double mu_o = (double)sx / (double)(2 * M);
  const double mu_s = (double)(sx + sf) / (double)(4 * M);
  const double am = aa * mu_o;
  a = aa;
  bb = mu_s - am;
  return kStNew;
}

// fit_sums of unit u = ((k * 2 + s) * NB + j) * 3 + c from the band sums in
// the caller layout.
__device__ inline int fit_new(const Geo& g, const uint64_t* band_sums, int u, double& a, double& bb) {
  const int nb = g.n_blocks;
  const int c = u % kCS;
  const int j = (u / kCS) % nb;
  const int s = (u / (kCS * nb)) & 1;
  const int k = u / (kCS * nb * 2);
  const DevCam& cam = g.cams[k];
  const int fc = cam.face_cam[s];
  const uint64_t* fac = fc < 0 ? nullptr : band_sums + unit_index(fc, cam.face_side[s], j, c, nb) * 3;
  return fit_sums(g, cam.channels, c, band_sums + (int64_t)u * 3, fac, a, bb);
}

// The state (p0, p1, v) of a unit after its fit, in place (section 3.1's
// exponential smoothing in smoothing mode; the first estimate is taken as is).
__device__ inline void temporal_step_mode(const Geo& g, int mode, int status, double a, double bb, double& p0,
                                          double& p1, uint8_t& v) {
  if (status == kStUnused || status == kStIdentity) {
    p0 = 1.0; p1 = 0.0; v = status == kStIdentity ? 1 : 0;
    return;
  }
  const bool had = v != 0;
  if (status == kStNone) {            // no estimate: keep the state
    if (!had) { p0 = 1.0; p1 = 0.0; }
    return;
  }
  if (mode == RT_MODE_SMOOTHING && had) {
    const double keep = 1.0 - g.alpha;
    const double ta = keep * p0;
    const double na = g.alpha * a;
    const double tb = keep * p1;
    const double nbv = g.alpha * bb;
    a = ta + na;
    bb = tb + nbv;
  }
  p0 = a;
  p1 = bb;
  v = 1;
}

// temporal_step_mode in the context's temporal mode.
__device__ inline void temporal_step(const Geo& g, int status, double a, double bb, double& p0, double& p1,
                                     uint8_t& v) {
  temporal_step_mode(g, g.mode, status, a, bb, p0, p1, v);
}

// Object removal with the smoothing fallback (section 3.1; section 4.1
// prefers removal when enough of a block remains).  Method of a seam unit
// from the channel-0 counts of the whole bands (own, fac) and of their kept
// pixels (kown, kfac): removal when both bands keep at least min_kept of
// their pixels (fractions in binary64), the smoothing fallback otherwise,
// none without a facing band or with an empty band.  Both sides of a seam
// see the same two fractions.
enum { kMethodNone = 0, kMethodRemoval = 1, kMethodSmoothing = 2 };

__device__ inline int removal_method(const uint64_t* own, const uint64_t* fac, const uint64_t* kown,
                                     const uint64_t* kfac, double min_kept) {
  if (!fac || own[0] == 0 || fac[0] == 0) return kMethodNone;
  const double fo = (double)kown[0] / (double)own[0];
  const double ff = (double)kfac[0] / (double)fac[0];
  return (kown[0] > 0 && kfac[0] > 0 && fo >= min_kept && ff >= min_kept) ? kMethodRemoval : kMethodSmoothing;
}

// Fit and state step of channel c of a unit under the method m: the removal
// fit from the kept sums in the context's mode, the fallback from the whole
// bands' sums, always smoothed (the first estimate taken as is).  own/fac and
// kown/kfac point at channel c's (n, S1, S2); fac and kfac NULL without a
// facing band.
__device__ inline void removal_step(const Geo& g, int m, int channels, int c, const uint64_t* own,
                                    const uint64_t* fac, const uint64_t* kown, const uint64_t* kfac, double& p0,
                                    double& p1, uint8_t& v) {
  double a, bb;
  const bool kept = m == kMethodRemoval;
  const int st = fit_sums(g, channels, c, kept ? kown : own, kept ? kfac : fac, a, bb);
  temporal_step_mode(g, m == kMethodSmoothing ? (int)RT_MODE_SMOOTHING : g.mode, st, a, bb, p0, p1, v);
}

// temporal_step on the state of unit u in the caller's buffers.
__device__ inline void temporal_update(const Geo& g, double* params, uint8_t* valid, int u, int status, double a,
                                       double bb) {
  double* p = params + (int64_t)u * 2;
  double p0 = p[0], p1 = p[1];
  uint8_t v = valid[u];
  temporal_step(g, status, a, bb, p0, p1, v);
  p[0] = p0;
  p[1] = p1;
  valid[u] = v;
}

// Fit and state update of unit u from the caller's buffers.
__device__ inline void estimate_unit(const Geo& g, const Bufs& b, int u) {
  double a, bb;
  const int st = fit_new(g, b.band_sums, u, a, bb);
  temporal_update(g, b.params, b.valid, u, st, a, bb);
}

// Entry x of the three channel tables of unit (k, s, j) = `unit3` (the
// channel-0 unit index divided by 3) from the maps ab[c] = (a, b); thread
// x == 0 also stores the q16 pairs.
__device__ inline void lut_entry_ab(const Geo& g, const Bufs& b, int unit3, int x, const double (*ab)[2]) {
  const int k = unit3 / (2 * g.n_blocks);
  const DevCam& cam = g.cams[k];
#pragma unroll
  for (int c = 0; c < kCS; ++c) {
    const int64_t u = (int64_t)unit3 * kCS + c;
    const int64_t A = (int64_t)__builtin_rint(ab[c][0] * 65536.0);
    const int64_t Bq = (int64_t)__builtin_rint(ab[c][1] * 65536.0);
    if (x == 0) {
      b.q16[u * 2 + 0] = A;
      b.q16[u * 2 + 1] = Bq;
    }
    if (cam.bps == 1) {
      int64_t y = (A * x + Bq + 32768) >> 16;
      y = y < 0 ? 0 : (y > 255 ? 255 : y);
      b.lut8[u * kNB + x] = (uint8_t)y;
    }
  }
}

// lut_entry_ab with the maps read from the caller's parameters.
__device__ inline void lut_entry(const Geo& g, const Bufs& b, int unit3, int x) {
  double ab[kCS][2];
#pragma unroll
  for (int c = 0; c < kCS; ++c) {
    const int64_t u = (int64_t)unit3 * kCS + c;
    ab[c][0] = b.params[u * 2 + 0];
    ab[c][1] = b.params[u * 2 + 1];
  }
  lut_entry_ab(g, b, unit3, x, ab);
}

// Q8 blend weight of column col of a camera of width W: h = floor(W/2); the
// left half has round_half_up(256 (h - col) / h), the right half its mirror,
// the centre column of an odd width 0.
__device__ inline uint32_t blend_weight(int W, int col) {
  const int h = W >> 1;
  if (col < h) return (uint32_t)(((h - col) * 256 + (h >> 1)) / h);
  if (col >= W - h && col < W) return (uint32_t)(((col - W + h + 1) * 256 + (h >> 1)) / h);
  return 0u;
}

}  // namespace rc
