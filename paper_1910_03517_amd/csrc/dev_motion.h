// Object removal of section 3.1 as device functions: the band statistics of
// one (camera, side, block) unit together with the sums of the band pixels
// that do not move, a pixel moving when its thresholded absolute difference
// to the previous frame exceeds the threshold on some channel.
#pragma once

#include "dev_stats.h"

namespace rc {

// Previous frames of a launch (device pointers; all NULL: nothing moves).
struct PrevPtrs {
  const uint8_t* in[RT_MAX_CAMS];
};

// Object-removal arguments of a launch.
struct Removal {
  uint64_t* kept_sums;   // [K][2][NB][3][3] (n, S1, S2) of the kept pixels
  uint8_t* method;       // [K][2][NB] method taken by each unit (may be NULL)
  int32_t tau;           // threshold in 8-bit units
  int32_t has_prev;      // 0: no previous frames, every pixel is kept
  double min_kept;       // least kept fraction of both bands for the removal fit
};

struct MotionLds {
  uint32_t hist[kCS * kNB];
  unsigned long long red[16 * 16];
};

// Barriers that band_unit_motion passes, on every path.
constexpr int kMotionBarriers = 4;

// Dword at byte offset boff of a row, bytes at or beyond row_bytes read as
// zero (a row's padding is never read).
__device__ inline uint32_t row_dword(__amdgpu_buffer_rsrc_t r, int rowoff, int boff, int row_bytes) {
  if (boff + 4 <= row_bytes) return __builtin_amdgcn_raw_buffer_load_b32(r, rowoff + boff, 0, 0);
  uint32_t d = 0;
  for (int e = 0; boff + e < row_bytes; ++e)
    d |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, rowoff + boff + e, 0, 0) << (8 * e);
  return d;
}

// The ND dwords of a row starting at byte offset o (any alignment): aligned
// loads, then byte shifts across neighbouring dwords.
template <int ND>
__device__ inline void group_dwords(__amdgpu_buffer_rsrc_t r, int rowoff, int o, int row_bytes, uint32_t (&w)[ND]) {
  const int base = o & ~3, sh = o & 3;
  uint32_t d[ND + 1];
#pragma unroll
  for (int i = 0; i <= ND; ++i) d[i] = (i < ND || sh) ? row_dword(r, rowoff, base + 4 * i, row_bytes) : 0u;
#pragma unroll
  for (int i = 0; i < ND; ++i) w[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], (uint32_t)sh);
}

// Sample i (0 .. 4 C - 1 in pixel-major order) of a group of 4 pixels.
template <int BPS>
__device__ inline uint32_t group_sample(const uint32_t* w, int i) {
  if (BPS == 1) return (w[i >> 2] >> (8 * (i & 3))) & 0xffu;
  return (w[i >> 1] >> (16 * (i & 1))) & 0xffffu;
}

// Band statistics of unit (k, s, j) (histogram and (n, S1, S2) of the whole
// band, written to the caller's band buffers as band_unit writes them) and
// the (n, S1, S2) of its kept pixels into rm.kept_sums.  kThreads threads
// (tid: the thread's index among them) walk the band in groups of 4 pixels.
// sums_out / kept_out (may be NULL) receive the nine whole-band and the
// nine kept sums of the unit as well.
template <int C, int BPS>
__device__ __attribute__((always_inline)) void band_unit_motion(const Geo& g, const FramePtrs& fp,
                                                                const PrevPtrs& pp, const Bufs& b,
                                                                const Removal& rm, int k, int s, int j,
                                                                MotionLds& L, uint64_t* sums_out,
                                                                uint64_t* kept_out, int tid) {
  constexpr int ND = C * BPS;                 // dwords of a 4-pixel group
  const DevCam cam = uniform_cam(g.cams[k]);
  for (int i = tid; i < kCS * kNB; i += kThreads) L.hist[i] = 0;
  __syncthreads();

  const int r0 = (int)((int64_t)j * cam.height / g.n_blocks);
  const int r1 = (int)((int64_t)(j + 1) * cam.height / g.n_blocks);
  const int band = cam.band;
  const int c0 = (s == 0) ? 0 : cam.width - band;
  const int ng = (band + 3) >> 2;             // groups per band row
  const int total = (r1 - r0) * ng;
  const int shift = cam.bit_depth - 8;
  const uint32_t thr = (uint32_t)rm.tau << shift;
  const bool has_prev = rm.has_prev != 0;
  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[k], cam);
  const __amdgpu_buffer_rsrc_t rprev = has_prev ? frame_rsrc(pp.in[k], cam) : rin;
  unsigned long long a1 = 0, a2 = 0;          // whole-band 16-bit sums
  unsigned long long kn = 0, k1[3] = {0, 0, 0}, k2[3] = {0, 0, 0};

  for (int idx = tid; idx < total; idx += kThreads) {
    const int row = idx / ng;
    const int q = idx - row * ng;
    const int rowoff = (int)((int64_t)(r0 + row) * cam.pitch);
    const int o = (c0 + 4 * q) * C * BPS;
    uint32_t w[ND], v[ND];
    group_dwords<ND>(rin, rowoff, o, cam.row_bytes, w);
    if (has_prev) group_dwords<ND>(rprev, rowoff, o, cam.row_bytes, v);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (4 * q + p >= band) continue;
      uint32_t x[C];
      bool moving = false;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        x[c] = group_sample<BPS>(w, p * C + c);
        if (has_prev) {
          const uint32_t y = group_sample<BPS>(v, p * C + c);
          const uint32_t d = x[c] > y ? x[c] - y : y - x[c];
          moving = moving || d > thr;
        }
        uint32_t bin = x[c];
        if (BPS == 2) {
          bin >>= shift;
          bin = bin > 255u ? 255u : bin;
          a1 += x[c];
          a2 += (unsigned long long)x[c] * x[c];
        }
        __hip_atomic_fetch_add(&L.hist[c * kNB + bin], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (!moving) {
        ++kn;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          k1[c] += x[c];
          k2[c] += (unsigned long long)x[c] * x[c];
        }
      }
    }
  }
  __syncthreads();

  const int64_t u0 = unit_index(k, s, j, 0, g.n_blocks);
  uint32_t* oh = b.band_hist + u0 * kNB;
  for (int i = tid; i < kCS * kNB; i += kThreads) oh[i] = L.hist[i];
  // Quantities 0..8: (n, S1, S2) of the whole band per channel slot (8-bit
  // sums from the exact histogram, thread tid holding bin tid); 9: kept n;
  // 10..12: kept S1 per channel slot; 13..15: kept S2.
  const unsigned long long x = (unsigned long long)tid;
  block_sums(
      16,
      [&](int i) -> unsigned long long {
        if (i < 9) {
          const int c = i / 3, m = i - 3 * (i / 3);
          if (c >= C) return 0ull;
          const unsigned long long h = L.hist[c * kNB + tid];
          if (m == 0) return h;
          if (BPS == 2) return m == 1 ? a1 : a2;
          return m == 1 ? h * x : h * x * x;
        }
        if (i == 9) return kn;
        const int c = (i - 10) % 3;
        if (c >= C) return 0ull;
        // (selected, not indexed: a run-time index would put the arrays in scratch)
        const unsigned long long s1 = c == 0 ? k1[0] : (c == 1 ? k1[1] : k1[2]);
        const unsigned long long s2 = c == 0 ? k2[0] : (c == 1 ? k2[1] : k2[2]);
        return i < 13 ? s1 : s2;
      },
      [&](int i, unsigned long long tot) {
        if (i < 9) {
          b.band_sums[u0 * 3 + i] = tot;
          if (sums_out) sums_out[i] = tot;
          return;
        }
        // Kept sums in the per-channel layout, n repeated for every channel
        // of the camera (zero for unused slots).
        uint64_t* ko = rm.kept_sums + u0 * 3;
        if (i == 9) {
#pragma unroll
          for (int c = 0; c < kCS; ++c) {
            const uint64_t n = c < C ? (uint64_t)tot : 0ull;
            ko[c * 3] = n;
            if (kept_out) kept_out[c * 3] = n;
          }
        } else {
          const int c = (i - 10) % 3, m = i < 13 ? 1 : 2;
          ko[c * 3 + m] = tot;
          if (kept_out) kept_out[c * 3 + m] = tot;
        }
      },
      L.red, tid);
}

// band_unit_motion of unit (camera, side, block) = `unit` (tid: the thread's
// index among the kThreads that take it).
__device__ __attribute__((always_inline)) inline void band_unit_motion_dispatch(
    const Geo& g, const FramePtrs& fp, const PrevPtrs& pp, const Bufs& b, const Removal& rm, int unit,
    MotionLds& L, uint64_t* sums_out, uint64_t* kept_out, int tid) {
  const int nb = g.n_blocks;
  const int k = unit / (2 * nb);
  const int s = (unit / nb) & 1;
  const int j = unit % nb;
  const DevCam& cam = g.cams[k];
  if (!cam_active(g, k)) return;
  if (cam.bps == 2) band_unit_motion<1, 2>(g, fp, pp, b, rm, k, s, j, L, sums_out, kept_out, tid);
  else if (cam.channels == 3) band_unit_motion<3, 1>(g, fp, pp, b, rm, k, s, j, L, sums_out, kept_out, tid);
  else band_unit_motion<1, 1>(g, fp, pp, b, rm, k, s, j, L, sums_out, kept_out, tid);
}

}  // namespace rc
