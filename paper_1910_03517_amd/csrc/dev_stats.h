// Statistics of section 3.1 as device functions: the band statistics of one
// (camera, side, block) unit, and the clearing of the whole-frame statistics
// that the apply pass accumulates.
#pragma once

#include "dev_common.h"

namespace rc {

struct StatsLds {
  uint32_t hist[kCS * kNB];
  unsigned long long red[9 * 16];
};

// Band statistics of unit (k, s, j): histogram and exact (n, S1, S2) of the
// band's samples.  Threads walk the band as (row, dword) pairs; a dword holds 4
// consecutive 8-bit samples or 2 16-bit samples of the row, and only the bytes
// inside the band count.  8-bit sums follow from the exact histogram.
// Barriers (__syncthreads) that band_unit passes, on every path.
constexpr int kBandBarriers = 4;

// (Inlined: an outlined call would take the kernel's by-value arguments by
// address, in scratch memory.)
template <int C, int BPS>
__device__ __attribute__((always_inline)) void band_unit(const Geo& g, const FramePtrs& fp, const Bufs& b, int k,
                                                         int s, int j, StatsLds& L, uint64_t* sums_out, int tid) {
  const DevCam cam = uniform_cam(g.cams[k]);
  auto clear = [&]() {
    for (int i = tid; i < kCS * kNB; i += kThreads) L.hist[i] = 0;
    __syncthreads();
  };

  const int r0 = (int)((int64_t)j * cam.height / g.n_blocks);
  const int r1 = (int)((int64_t)(j + 1) * cam.height / g.n_blocks);
  const int band = cam.band;
  const int c0 = (s == 0) ? 0 : cam.width - band;
  const int b0 = c0 * C * BPS;                 // band bytes [b0, b1) of each row
  const int b1 = (c0 + band) * C * BPS;
  const int q0 = b0 >> 2;
  const int dw = ((b1 + 3) >> 2) - q0;         // dwords per band row
  const int rows = r1 - r0;
  const int shift = cam.bit_depth - 8;
  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[k], cam);
  unsigned long long a1 = 0, a2 = 0;           // 16-bit sums

  // One sample (byte offset o of the row) into the histogram.
  auto count = [&](uint32_t d, int boff) {
    if (BPS == 1) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = boff + e;
        if (o >= b0 && o < b1) {
          const uint32_t v = (d >> (8 * e)) & 0xffu;
          const int c = (C == 1) ? 0 : o % C;
          __hip_atomic_fetch_add(&L.hist[c * kNB + v], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int o = boff + 2 * e;
        if (o >= b0 && o < b1) {
          const uint32_t v = (d >> (16 * e)) & 0xffffu;
          uint32_t bin = v >> shift;
          bin = bin > 255u ? 255u : bin;
          __hip_atomic_fetch_add(&L.hist[bin], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          a1 += v;
          a2 += (unsigned long long)v * v;
        }
      }
    }
  };
  // A dword of the band row at byte offset boff; the one crossing the row end
  // is assembled from single bytes.
  auto load = [&](int rowoff, int boff) -> uint32_t {
    if (boff + 4 <= cam.row_bytes) return __builtin_amdgcn_raw_buffer_load_b32(rin, rowoff + boff, 0, 0);
    uint32_t d = 0;
    for (int e = 0; boff + e < cam.row_bytes; ++e)
      d |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rin, rowoff + boff + e, 0, 0) << (8 * e);
    return d;
  };

  constexpr int kU = 4;                        // loads in flight per thread
  if (band > 0 && rows > 0 && dw <= kThreads) {
    // Thread tid keeps one dword column q of the band and walks the rows
    // tid / dw, + rstep, ...: no division per load.
    const int rstep = kThreads / dw;
    const int q = tid % dw;
    const int boff = (q0 + q) * 4;
    constexpr int kR = 2 * kU;                 // a 67-row block of a 32-pixel RGB band in one round
    const bool active = tid < rstep * dw;
    uint32_t d[kR];
    auto fetch = [&](int row) {
#pragma unroll
      for (int u = 0; u < kR; ++u) {
        const int r = row + u * rstep;
        d[u] = r < rows ? load((int)((int64_t)(r0 + r) * cam.pitch), boff) : 0u;
      }
    };
    // The first round of loads is in flight while the histogram is cleared.
    if (active) fetch(tid / dw);
    clear();
    if (active) {
      for (int row = tid / dw; row < rows; row += kR * rstep) {
        if (row != tid / dw) fetch(row);
#pragma unroll
        for (int u = 0; u < kR; ++u)
          if (row + u * rstep < rows) count(d[u], boff);
      }
    }
  } else if (band > 0 && rows > 0) {
    clear();
    const int total = rows * dw;
    for (int base = tid; base < total; base += kU * kThreads) {
      uint32_t d[kU];
      int boffs[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int idx = base + u * kThreads;
        d[u] = 0;
        boffs[u] = -1;
        if (idx < total) {
          const int row = idx / dw;
          const int q = idx - row * dw;
          boffs[u] = (q0 + q) * 4;
          d[u] = load((int)((int64_t)(r0 + row) * cam.pitch), boffs[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (boffs[u] >= 0) count(d[u], boffs[u]);
    }
  } else {
    clear();
  }
  __syncthreads();

  const int64_t u0 = unit_index(k, s, j, 0, g.n_blocks);
  uint32_t* oh = b.band_hist + u0 * kNB;
  for (int i = tid; i < kCS * kNB; i += kThreads) oh[i] = L.hist[i];
  // (n, S1, S2) per channel slot: quantity i is channel i / 3, moment i % 3.
  const unsigned long long x = (unsigned long long)tid;
  block_sums(
      9,
      [&](int i) -> unsigned long long {
        const int c = i / 3, m = i - 3 * (i / 3);
        if (c >= C) return 0ull;
        const unsigned long long h = L.hist[c * kNB + tid];
        if (m == 0) return h;
        if (BPS == 2) return m == 1 ? a1 : a2;
        return m == 1 ? h * x : h * x * x;
      },
      [&](int i, unsigned long long tot) {
        b.band_sums[u0 * 3 + i] = tot;
        if (sums_out) sums_out[i] = tot;
      },
      L.red, tid);
}

// Band statistics of unit (camera, side, block) = `unit` by kThreads threads
// (tid: the thread's index among them; -1: the workgroup's threadIdx.x); with
// sums_out (LDS) its nine sums are also left there for the workgroup.
__device__ __attribute__((always_inline)) inline void band_unit_dispatch(const Geo& g, const FramePtrs& fp,
                                                                         const Bufs& b, int unit, StatsLds& L,
                                                                         uint64_t* sums_out = nullptr,
                                                                         int tid = -1) {
  if (tid < 0) tid = (int)threadIdx.x;
  const int nb = g.n_blocks;
  const int k = unit / (2 * nb);
  const int s = (unit / nb) & 1;
  const int j = unit % nb;
  const DevCam& cam = g.cams[k];
  if (!cam_active(g, k)) return;
  if (cam.bps == 2) band_unit<1, 2>(g, fp, b, k, s, j, L, sums_out, tid);
  else if (cam.channels == 3) band_unit<3, 1>(g, fp, b, k, s, j, L, sums_out, tid);
  else band_unit<1, 1>(g, fp, b, k, s, j, L, sums_out, tid);
}

// Zero the whole-frame histogram and sums of every active camera (grid-stride).
__device__ inline void zero_whole(const Geo& g, const Bufs& b, int thread, int nthreads) {
  const int nh = g.n_cams * kCS * kNB;
  for (int i = thread; i < nh; i += nthreads)
    if (cam_active(g, i / (kCS * kNB))) b.whole_hist[i] = 0u;
  for (int i = thread; i < g.n_cams * 9; i += nthreads)
    if (cam_active(g, i / 9)) b.whole_sums[i] = 0ull;
}

}  // namespace rc
