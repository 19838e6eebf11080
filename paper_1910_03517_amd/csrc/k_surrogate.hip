// Learned surrogate of the estimate, per (camera, side, block) unit of the
// RGB cameras: its 576 input features, the plain estimate before the temporal
// step (which judges the network and is the fallback), the training targets,
// and the per-unit choice between network and plain estimate followed by the
// temporal update of the estimator state.
#include "dev_estimate.h"
#include "dev_stats.h"
#include "dev_mlp.h"

namespace rc {

// Features of unit u3 = (k * 2 + s) * NB + j: regions (whole frame of camera k
// as given, own band, facing band), channels, 64 bins = 64 * (sum of 4
// adjacent 256-bins) / the region-channel's count, computed in binary64 and
// rounded once to float32.  Rows of non-RGB cameras are zero.
// Features of unit u3 (one workgroup): wave w takes the region-channel pairs
// rc = w, w + 4, w + 8 (rc = 3 r + c, features rc * 64 .. rc * 64 + 63); lane
// l holds bin l's four 256-bins, and the pair's count is the wave's sum.
__device__ __forceinline__ void features_unit(const Geo& g, const uint32_t* __restrict__ band_hist,
                                              const uint32_t* __restrict__ whole_hist, float* __restrict__ X,
                                              int u3) {
  const int nb = g.n_blocks;
  const int k = u3 / (2 * nb);
  const int s = (u3 / nb) & 1;
  const int j = u3 % nb;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const DevCam& cam = g.cams[k];
  float* out = X + (int64_t)u3 * kMlpIn;
  if (cam.channels != 3) {
    for (int o = tid; o < kMlpIn; o += kThreads) out[o] = 0.0f;
    return;
  }
  const int fc = cam.face_cam[s];
  const uint32_t* base[3] = {whole_hist + (int64_t)k * kCS * kNB, band_hist + unit_index(k, s, j, 0, nb) * kNB,
                             fc >= 0 ? band_hist + unit_index(fc, cam.face_side[s], j, 0, nb) * kNB : nullptr};
  for (int rc = tid / kWave; rc < 3 * kCS; rc += kThreads / kWave) {
    const uint32_t* h = base[rc / kCS];
    uint32_t m = 0;
    if (h) {
      h += (rc % kCS) * kNB + 4 * lane;
      m = h[0] + h[1] + h[2] + h[3];
    }
    const unsigned long long n = wave_sum_u64(m);
    out[rc * 64 + lane] = n ? (float)((double)m * 64.0 / (double)n) : 0.0f;
  }
}

__global__ __launch_bounds__(kThreads) void k_features(Geo g, const uint32_t* __restrict__ band_hist,
                                                       const uint32_t* __restrict__ whole_hist, float* __restrict__ X) {
  const int u3 = blockIdx.x;
  if (!cam_active(g, u3 / (2 * g.n_blocks))) return;
  features_unit(g, band_hist, whole_hist, X, u3);
}

// The plain estimate of every (camera, side, block, channel) before the temporal step.
__global__ __launch_bounds__(kThreads) void k_estimate_new(Geo g, const uint64_t* __restrict__ band_sums,
                                                           double* __restrict__ p_new, int32_t* __restrict__ status) {
  const int u = blockIdx.x * kThreads + threadIdx.x;
  if (u >= g.n_cams * 2 * g.n_blocks * kCS || !cam_active(g, u / (2 * g.n_blocks * kCS))) return;
  double a, b;
  status[u] = fit_new(g, band_sums, u, a, b);
  p_new[(int64_t)u * 2] = a;
  p_new[(int64_t)u * 2 + 1] = b;
}

// Training targets (a_R, a_G, a_B, b_R/255, b_G/255, b_B/255) of every unit,
// and mask[u3] = 1 where the unit is RGB and all three channels hold a new estimate.
__global__ __launch_bounds__(kThreads) void k_targets(Geo g, const double* __restrict__ p_new,
                                                      const int32_t* __restrict__ status, float* __restrict__ T,
                                                      uint8_t* __restrict__ mask) {
  const int u3 = blockIdx.x * kThreads + threadIdx.x;
  if (u3 >= g.n_cams * 2 * g.n_blocks) return;
  const int k = u3 / (2 * g.n_blocks);
  bool ok = g.cams[k].channels == 3;
  for (int c = 0; c < kCS; ++c) {
    const int64_t u = (int64_t)u3 * kCS + c;
    ok = ok && status[u] == kStNew;
    T[(int64_t)u3 * kMlpOut + c] = (float)p_new[u * 2];
    T[(int64_t)u3 * kMlpOut + 3 + c] = (float)(p_new[u * 2 + 1] / 255.0);
  }
  mask[u3] = ok ? 1 : 0;
}

// Per unit: take the network's prediction iff the unit is RGB, all three
// channels hold a new plain estimate, every output is finite and
// r = max_c max(|a^ - a|, |b^n - b / 255|) <= tol (binary64 on the float32
// outputs); then the temporal update of the three channels.
__device__ inline void select_unit(const Geo& g, const float* __restrict__ Y, const double* __restrict__ p_new,
                                   const int32_t* __restrict__ status, float tol, double* __restrict__ params,
                                   uint8_t* __restrict__ valid, uint8_t* __restrict__ used,
                                   float* __restrict__ residual, int u3) {
  const int k = u3 / (2 * g.n_blocks);
  const float* y = Y + (int64_t)u3 * kMlpOut;
  bool eligible = g.cams[k].channels == 3;
  for (int c = 0; c < kCS; ++c) eligible = eligible && status[(int64_t)u3 * kCS + c] == kStNew;
  bool finite = true;
  for (int o = 0; o < kMlpOut; ++o) finite = finite && __builtin_isfinite(y[o]);
  double r = __builtin_inf();
  if (eligible && finite) {
    r = 0.0;
    for (int c = 0; c < kCS; ++c) {
      const int64_t u = (int64_t)u3 * kCS + c;
      const double da = __builtin_fabs((double)y[c] - p_new[u * 2]);
      const double db = __builtin_fabs((double)y[3 + c] - p_new[u * 2 + 1] / 255.0);
      r = da > r ? da : r;
      r = db > r ? db : r;
    }
  }
  const bool use = eligible && finite && r <= (double)tol;
  used[u3] = use ? 1 : 0;
  residual[u3] = (float)r;
  for (int c = 0; c < kCS; ++c) {
    const int u = u3 * kCS + c;
    double a = p_new[(int64_t)u * 2], b = p_new[(int64_t)u * 2 + 1];
    if (use) {
      a = (double)y[c];
      b = 255.0 * (double)y[3 + c];
    }
    temporal_update(g, params, valid, u, status[u], a, b);
  }
}

__global__ __launch_bounds__(kThreads) void k_select(Geo g, const float* __restrict__ Y,
                                                     const double* __restrict__ p_new,
                                                     const int32_t* __restrict__ status, float tol,
                                                     double* __restrict__ params, uint8_t* __restrict__ valid,
                                                     uint8_t* __restrict__ used, float* __restrict__ residual) {
  const int u3 = blockIdx.x * kThreads + threadIdx.x;
  if (u3 >= g.n_cams * 2 * g.n_blocks) return;
  if (!cam_active(g, u3 / (2 * g.n_blocks))) return;
  select_unit(g, Y, p_new, status, tol, params, valid, used, residual, u3);
}

// Surrogate frame-set, step 1 (one workgroup per unit u3): the unit's
// features, and its three channels' plain estimate (three lanes of the last wave).
__global__ __launch_bounds__(kThreads) void k_features_new(Geo g, const uint32_t* __restrict__ band_hist,
                                                           const uint64_t* __restrict__ band_sums,
                                                           const uint32_t* __restrict__ whole_hist,
                                                           float* __restrict__ X, double* __restrict__ p_new,
                                                           int32_t* __restrict__ status) {
  const int u3 = blockIdx.x;
  if (!cam_active(g, u3 / (2 * g.n_blocks))) return;
  const int tid = threadIdx.x - (kThreads - kWave);   // the last wave, which has the fewest feature pairs
  if (tid >= 0 && tid < kCS) {
    const int u = u3 * kCS + tid;
    double a, b;
    status[u] = fit_new(g, band_sums, u, a, b);
    p_new[(int64_t)u * 2] = a;
    p_new[(int64_t)u * 2 + 1] = b;
  }
  features_unit(g, band_hist, whole_hist, X, u3);
}

// Surrogate frame-set, step 3 (one workgroup per unit u3): the network's
// output row (wave 0, the routine of the forward pass's output layer), the
// choice and state update (thread 0, which stored that row), the unit's
// tables, the camera's weights (first unit), and clearing the whole-frame
// statistics the apply accumulates.
__global__ __launch_bounds__(kThreads) void k_select_lut(Geo g, const float* __restrict__ H2,
                                                         const float* __restrict__ W3, const float* __restrict__ b3,
                                                         float* __restrict__ Y, const double* __restrict__ p_new,
                                                         const int32_t* __restrict__ status, float tol, Bufs b,
                                                         uint8_t* __restrict__ used, float* __restrict__ residual) {
  const int u3 = blockIdx.x;
  const int tid = threadIdx.x;
  const int nb = g.n_blocks;
  const int k = u3 / (2 * nb);
  if (b.whole_hist) zero_whole(g, b, blockIdx.x * kThreads + tid, gridDim.x * kThreads);
  if (!cam_active(g, k)) return;
  if (tid < kWave) {
    float acc[kMlpOut];
    wave_row_dot<kMlpOut>(H2 + (int64_t)u3 * kMlpHid, W3, b3, kMlpHid, kMlpOut, acc);
    if (tid == 0) {
#pragma unroll
      for (int o = 0; o < kMlpOut; ++o) Y[(int64_t)u3 * kMlpOut + o] = acc[o];
      select_unit(g, Y, p_new, status, tol, b.params, b.valid, used, residual, u3);
    }
  }
  __syncthreads();
  lut_entry(g, b, u3, tid);
  if (u3 % (2 * nb) == 0)
    for (int col = tid; col < g.w_max; col += kThreads)
      b.weights[(int64_t)k * g.w_max + col] = (uint16_t)blend_weight(g.cams[k].width, col);
}

hipError_t launch_features(const Geo& g, const uint32_t* band_hist, const uint32_t* whole_hist, float* X,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, band_hist, whole_hist, X);
  return hipGetLastError();
}

hipError_t launch_estimate_new(const Geo& g, const uint64_t* band_sums, double* p_new, int32_t* status,
                               hipStream_t st) {
  const int n = g.n_cams * 2 * g.n_blocks * kCS;
  hipLaunchKernelGGL(k_estimate_new, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, band_sums, p_new,
                     status);
  return hipGetLastError();
}

hipError_t launch_targets(const Geo& g, const double* p_new, const int32_t* status, float* T, uint8_t* mask,
                          hipStream_t st) {
  const int n = g.n_cams * 2 * g.n_blocks;
  hipLaunchKernelGGL(k_targets, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, p_new, status, T, mask);
  return hipGetLastError();
}

hipError_t launch_features_new(const Geo& g, const uint32_t* band_hist, const uint64_t* band_sums,
                               const uint32_t* whole_hist, float* X, double* p_new, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_features_new, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, band_hist, band_sums,
                     whole_hist, X, p_new, status);
  return hipGetLastError();
}

hipError_t launch_select_lut(const Geo& g, const float* H2, const float* W3, const float* b3, float* Y,
                             const double* p_new, const int32_t* status, float tol, const Bufs& b, uint8_t* used,
                             float* residual, hipStream_t st) {
  hipLaunchKernelGGL(k_select_lut, dim3(g.n_cams * 2 * g.n_blocks), dim3(kThreads), 0, st, g, H2, W3, b3, Y, p_new,
                     status, tol, b, used, residual);
  return hipGetLastError();
}

hipError_t launch_select(const Geo& g, const float* Y, const double* p_new, const int32_t* status, float tol,
                         double* params, uint8_t* valid, uint8_t* used, float* residual, hipStream_t st) {
  const int n = g.n_cams * 2 * g.n_blocks;
  hipLaunchKernelGGL(k_select, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, Y, p_new, status, tol,
                     params, valid, used, residual);
  return hipGetLastError();
}

}  // namespace rc
