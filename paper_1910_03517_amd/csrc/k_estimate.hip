// Estimate and table kernels of section 3.1: shared spectrum at each seam,
// per-channel affine fit, exponential smoothing, fixed-point tables and the
// Q8 weights of the convex blend.  Binary64 throughout with contraction off,
// so every result is the correctly rounded value of the written expression.
#include "rt_internal.h"

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

// One thread per (camera, side, block, channel).  Both sides of a seam derive
// the same shared moments because binary64 addition is commutative.
__global__ __launch_bounds__(256) void k_estimate(Geo g, Bufs b) {
  const int nb = g.n_blocks;
  const int total = g.n_cams * 2 * nb * kCS;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= total) return;
  const int c = u % kCS;
  const int j = (u / kCS) % nb;
  const int s = (u / (kCS * nb)) & 1;
  const int k = u / (kCS * nb * 2);
  const DevCam& cam = g.cams[k];
  double* p = b.params + (int64_t)u * 2;
  if (c >= cam.channels) {
    p[0] = 1.0; p[1] = 0.0; b.valid[u] = 0;
    return;
  }
  const int fc = cam.face_cam[s];
  if (fc < 0) {                       // open chain end: identity
    p[0] = 1.0; p[1] = 0.0; b.valid[u] = 1;
    return;
  }
  const int64_t fu = unit_index(fc, cam.face_side[s], j, c, nb);
  const uint64_t* own = b.band_sums + (int64_t)u * 3;
  const uint64_t* fac = b.band_sums + fu * 3;
  const bool had = b.valid[u] != 0;
  if (own[0] == 0 || fac[0] == 0) {   // no estimate: keep the state
    if (!had) { p[0] = 1.0; p[1] = 0.0; }
    return;
  }
  const Moments mo = moments_of(own[0], own[1], own[2]);
  const Moments mf = moments_of(fac[0], fac[1], fac[2]);
  const double mu_s = (mo.mu + mf.mu) / 2.0;
  const double sd_s = (mo.sd + mf.sd) / 2.0;
  double a = (mo.var == 0.0) ? 1.0 : sd_s / mo.sd;
  a = a < g.a_min ? g.a_min : a;
  a = a > g.a_max ? g.a_max : a;
  const double am = a * mo.mu;
  double bb = mu_s - am;
  if (g.mode == RT_MODE_SMOOTHING && had) {
    const double keep = 1.0 - g.alpha;
    const double ta = keep * p[0];
    const double na = g.alpha * a;
    const double tb = keep * p[1];
    const double nbv = g.alpha * bb;
    a = ta + na;
    bb = tb + nbv;
  }
  p[0] = a;
  p[1] = bb;
  b.valid[u] = 1;
}

hipError_t launch_estimate(const Geo& g, const Bufs& b, hipStream_t st) {
  const int total = g.n_cams * 2 * g.n_blocks * kCS;
  hipLaunchKernelGGL(k_estimate, dim3((total + 255) / 256), dim3(256), 0, st, g, b);
  return hipGetLastError();
}

// One workgroup per (camera, side, block); thread x builds entry x of the
// three channel tables.  Thread 0 also stores the q16 pairs.
__global__ __launch_bounds__(256) void k_build_lut(Geo g, Bufs b) {
  const int unit = blockIdx.x;          // (k * 2 + s) * nb + j
  const int k = unit / (2 * g.n_blocks);
  const DevCam& cam = g.cams[k];
  const int x = threadIdx.x;
#pragma unroll
  for (int c = 0; c < kCS; ++c) {
    const int64_t u = (int64_t)unit * kCS + c;
    const double a = b.params[u * 2 + 0];
    const double bv = b.params[u * 2 + 1];
    const int64_t A = (int64_t)__builtin_rint(a * 65536.0);
    const int64_t Bq = (int64_t)__builtin_rint(bv * 65536.0);
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

// Q8 weights: one thread per (camera, column < w_max).
__global__ __launch_bounds__(256) void k_weights(Geo g, Bufs b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)g.n_cams * g.w_max) return;
  const int k = (int)(i / g.w_max);
  const int col = (int)(i - (int64_t)k * g.w_max);
  const int W = g.cams[k].width;
  const int h = W / 2;
  int w = 0;
  if (col < W) {
    if (col < h) w = ((h - col) * 256 + h / 2) / h;
    else if (col >= W - h) w = ((col - W + h + 1) * 256 + h / 2) / h;
  }
  b.weights[i] = (uint16_t)w;
}

hipError_t launch_build_lut(const Geo& g, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_build_lut, dim3(g.n_cams * 2 * g.n_blocks), dim3(256), 0, st, g, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)g.n_cams * g.w_max;
  hipLaunchKernelGGL(k_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace rc
