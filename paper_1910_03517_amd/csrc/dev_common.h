// Device helpers shared by the kernels: wave/block reductions.
#pragma once

#include "rt_internal.h"

namespace rc {

constexpr int kWave = 64;

// v moved by one DPP row operation (both 32-bit halves from the same source
// lane); lanes without a source lane, or outside row_mask, get 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline unsigned long long dpp_u64(unsigned long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROW_MASK, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROW_MASK, 0xf, false);
  return ((unsigned long long)hi << 32) | lo;
}

// Sum of v over the 64 lanes of the wave (all lanes active), returned to every
// lane.  Inclusive prefix sums within each row of 16 lanes (row_shr 1, 2, 4,
// 8), then the last lane of row 0 added to rows 1 and 3 (row_bcast:15) and the
// last lane of row 1 to rows 2 and 3 (row_bcast:31): lane 63 holds the total.
// DPP moves stay in the vector ALU, unlike lane shuffles through the LDS.
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  v += dpp_u64<0x111>(v);          // row_shr:1
  v += dpp_u64<0x112>(v);          // row_shr:2
  v += dpp_u64<0x114>(v);          // row_shr:4
  v += dpp_u64<0x118>(v);          // row_shr:8
  v += dpp_u64<0x142, 0xa>(v);     // row_bcast:15 into rows 1 and 3
  v += dpp_u64<0x143, 0xc>(v);     // row_bcast:31 into rows 2 and 3
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Sums over kThreads threads of n 64-bit quantities (n <= 16), one after
// the other to keep register pressure low: value(i) gives this thread's share
// of quantity i; thread i then receives the total as store(i, total).  `red`
// is LDS scratch of n * 16 words.  tid is the thread's index among the
// kThreads (the workgroup, or one part of a larger workgroup whose other
// parts make their own calls with their own `red`).  Contains two
// __syncthreads(): every wave of the workgroup must make the call.
template <typename Value, typename Store>
__device__ inline void block_sums(int n, Value value, Store store, unsigned long long* red, int tid) {
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

template <typename Value, typename Store>
__device__ inline void block_sums(int n, Value value, Store store, unsigned long long* red) {
  block_sums(n, value, store, red, (int)threadIdx.x);
}

}  // namespace rc
