// Device helpers of the surrogate network's kernels: a float wave sum and
// the output layer's per-row dot product, shared so that every kernel that
// computes the output layer produces the same bits.
#pragma once

#include "dev_common.h"
#include "rt_surrogate_internal.h"

namespace rc {

// Float sum of v over the 64 lanes of the wave (all lanes active) with the
// DPP steps of wave_sum_u64, in a fixed order; the total is returned to every lane.
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline float dpp_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                                                 false));
}
__device__ inline float wave_sum_f32(float v) {
  v += dpp_f32<0x111>(v);
  v += dpp_f32<0x112>(v);
  v += dpp_f32<0x114>(v);
  v += dpp_f32<0x118>(v);
  v += dpp_f32<0x142, 0xa>(v);
  v += dpp_f32<0x143, 0xc>(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// One output row of the network's last layer, y[o] = b[o] + sum_k h[k] w[k][o]
// for o < n_out <= 8 over K inputs, by one whole wave: lane l sums k = l,
// l + 64, ... and the wave adds the lanes.  Every caller of the last layer
// uses this one routine, so its results are the same bits wherever it runs.
template <int NMAX>
__device__ inline void wave_row_dot(const float* __restrict__ h, const float* __restrict__ w,
                                    const float* __restrict__ bias, int K, int n_out, float* acc) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 0; o < NMAX; ++o) acc[o] = 0.0f;
  for (int k = lane; k < K; k += kWave) {
    const float a = h ? h[k] : 1.0f;
#pragma unroll
    for (int o = 0; o < NMAX; ++o)
      if (o < n_out) acc[o] += a * w[(int64_t)k * n_out + o];
  }
#pragma unroll
  for (int o = 0; o < NMAX; ++o) {
    acc[o] = wave_sum_f32(acc[o]);
    if (bias && o < n_out) acc[o] += bias[o];
  }
}

}  // namespace rc
