// Device helpers shared by the kernels: wave/block reductions.
#pragma once

#include "rt_internal.h"

namespace rc {

constexpr int kWave = 64;

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int m = kWave / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// Workgroup sums of n 64-bit quantities (n <= 16), one after the other to
// keep register pressure low: value(i) gives this thread's share of quantity
// i; thread i then receives the total as store(i, total).  `red` is LDS
// scratch of n * 16 words.  Contains __syncthreads(): call from uniform
// control flow with blockDim.x == kThreads.
template <typename Value, typename Store>
__device__ inline void block_sums(int n, Value value, Store store, unsigned long long* red) {
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
#pragma unroll 1
  for (int i = 0; i < n; ++i) {
    const unsigned long long s = wave_sum_u64(value(i));
    if (lane == 0) red[i * 16 + wave] = s;
  }
  __syncthreads();
  if (tid < n) {
    unsigned long long s = 0;
    for (int w = 0; w < kThreads / kWave; ++w) s += red[tid * 16 + w];
    store(tid, s);
  }
  __syncthreads();
}

}  // namespace rc
