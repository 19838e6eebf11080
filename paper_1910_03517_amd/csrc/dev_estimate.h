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
