// Apply pass of section 3.1 as device functions over segments of rows: every
// sample is blended between the identity and its side's affine map with the
// Q8 weight of its column, y = ((256 - w) x + w f(x) + 128) >> 8, in exact
// integers; optionally fused with the whole-frame histogram and sums of the
// input samples.
//
// A thread owns groups of 4 consecutive pixels of a row (12 bytes for RGB8, 4
// for gray8, 8 for gray16) and walks down its segments' rows, kUnroll rows at
// a time so that several loads are in flight; its pixels' weights and map
// constants stay in registers.  The histogram is kept in LDS in kRep replicas
// interleaved bin by bin, lane l updating replica l % kRep, so that lanes of
// one wave that see the same value mostly hit different LDS words (packed
// variants, two 16-bit bins per word, are compile-time options; the segment
// tables then bound the rows between flushes so that no half can reach
// 2^16).  After a workgroup's last segment of a camera the replicas are summed
// and added to the camera's whole-frame statistics with global atomics (the
// whole-frame buffers must be zero before the first segment).
#pragma once

#include "dev_estimate.h"
#include "dev_stats.h"

namespace rc {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));

#ifndef RC_APPLY_UNROLL
#define RC_APPLY_UNROLL 6     // measured on MI355X: best when applies of consecutive frame-sets overlap
#endif
#ifndef RC_APPLY_DIRECT
#define RC_APPLY_DIRECT 1     // evaluate 8-bit maps from their Q16 pairs instead of the LDS tables
#endif
#ifndef RC_LOAD_POLICY
#define RC_LOAD_POLICY 2      // non-temporal: every frame byte is touched exactly once
#endif
#ifndef RC_STORE_POLICY
#define RC_STORE_POLICY 2
#endif
constexpr bool kPack = RC_APPLY_PACK != 0;  // two 16-bit bins per histogram word
constexpr int kRep = RC_APPLY_REP;        // histogram replicas
constexpr int kHistWords = kCS * (kPack ? kNB / 2 : kNB) * kRep;
constexpr int kUnroll = RC_APPLY_UNROLL;  // rows in flight per thread
constexpr int kLoadPolicy = RC_LOAD_POLICY;    // cache-policy bits of frame loads
constexpr int kStorePolicy = RC_STORE_POLICY;  // cache-policy bits of frame stores

// Word (before the replica index) and bit offset of (channel c, bin) in the
// LDS histogram.  Unpacked: a word per bin.  RC_APPLY_PACK 1: bins 2i and
// 2i + 1 share word i; RC_APPLY_PACK 2: bins i and i + 128 share word i, so
// that neighbouring values, frequent within a region, fall in different words.
__device__ inline int hist_word(int c, uint32_t bin) {
  if (RC_APPLY_PACK == 1) return c * (kNB / 2) + (int)(bin >> 1);
  if (RC_APPLY_PACK == 2) return c * (kNB / 2) + (int)(bin & (kNB / 2 - 1));
  return c * kNB + (int)bin;
}
__device__ inline uint32_t hist_shift(uint32_t bin) {
  if (RC_APPLY_PACK == 1) return (bin & 1u) << 4;
  if (RC_APPLY_PACK == 2) return (bin >> 7) << 4;
  return 0u;
}

struct ApplyLds {
  uint8_t lut[2 * kCS * kNB];          // [side][channel][x]
  int64_t q[4];                        // [side][A, Bq]
  uint32_t hist[kHistWords];           // [channel][bin (pair when packed)][replica]
  unsigned long long red[9 * 16];
};

template <int NW, int POL = kLoadPolicy>
__device__ inline void load_group(__amdgpu_buffer_rsrc_t r, int off, uint32_t (&d)[NW]) {
  if constexpr (NW == 3) {
    u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, POL);
    d[0] = v.x; d[1] = v.y; d[2] = v.z;
  } else if constexpr (NW == 2) {
    u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, POL);
    d[0] = v.x; d[1] = v.y;
  } else {
    d[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, POL);
  }
}

template <int NW, int POL = kStorePolicy>
__device__ inline void store_group(__amdgpu_buffer_rsrc_t r, int off, const uint32_t (&d)[NW]) {
  if constexpr (NW == 3) {
    u32x3 v = {d[0], d[1], d[2]};
    __builtin_amdgcn_raw_buffer_store_b96(v, r, off, 0, POL);
  } else if constexpr (NW == 2) {
    u32x2 v = {d[0], d[1]};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, POL);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(d[0], r, off, 0, POL);
  }
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per-pixel constants of a thread's group.
struct PixConst {
  uint32_t wp[4];         // Q8 weight pair: (256 - w) in the low half, w in the high half
  int lb[4];              // table base of the pixel's side
  int64_t qa[4], qb[4];   // 16-bit map of the pixel's side
  int32_t da[4][3];       // direct 8-bit map of the pixel's side: A and Bq + 2^15 per channel
  int32_t dc[4][3];
};

// The 8-bit table entry f(x) = clamp((A x + Bq + 2^15) >> 16, 0, 255) can be
// evaluated directly in 32-bit integers, bit for bit equal to the table, when
// |A| < 2^23 (a 24-bit multiply) and A x + Bq + 2^15 stays inside int32 for
// x in [0, 255].  The check is made once per segment on its six (A, Bq) pairs.
__device__ inline bool direct_ok(int64_t A, int64_t Bq) {
  if (A >= (1 << 23) || A < -(1 << 23)) return false;
  const int64_t c = Bq + 32768, e = 255 * A + c;
  const int64_t lo = c < e ? c : e, hi = c < e ? e : c;
  return lo >= INT32_MIN && hi <= INT32_MAX;
}

// Returns the blended sample, or with RAW the dot product itself: the sample
// is then its byte 1 and bytes 2-3 are zero (the sum stays below 2^16).
template <int BPS, bool WRITE, bool STATS, bool DIRECT = false, bool RAW = false>
__device__ inline uint32_t one_sample(uint32_t x, int c, int p, const PixConst& pc, ApplyLds& L, int hrep,
                                      int shift, uint32_t maxv, unsigned long long& a1, unsigned long long& a2) {
  if (STATS) {
    uint32_t bin = x;
    if (BPS == 2) { bin = x >> shift; bin = bin > 255u ? 255u : bin; }
    __hip_atomic_fetch_add(&L.hist[hist_word(c, bin) * kRep + hrep], 1u << hist_shift(bin), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    if (BPS == 2) { a1 += x; a2 += (unsigned long long)x * x; }
  }
  if (!WRITE) return 0;
  uint32_t f, xf;
  if (BPS == 1 && DIRECT) {
    // da holds a sign-extended 24-bit value (see direct_ok), so this is a 24-bit multiply.
    // clamp(v >> 16, 0, 255) << 16 == clamp(v, 0, 2^24 - 1) & 0xffff0000 for the
    // arithmetic shift, so f lands in the high half of (x, f) directly.
    const int32_t a24 = (int32_t)((uint32_t)pc.da[p][c] << 8) >> 8;
    int32_t v = a24 * (int32_t)x + pc.dc[p][c];
    v = v < 0 ? 0 : (v > 0xffffff ? 0xffffff : v);
    xf = ((uint32_t)v & 0xffff0000u) | x;
  } else if (BPS == 1) {
    f = L.lut[pc.lb[p] + c * kNB + x];
  } else {
    int64_t y = (pc.qa[p] * (int64_t)x + pc.qb[p] + 32768) >> 16;
    y = y < 0 ? 0 : (y > (int64_t)maxv ? (int64_t)maxv : y);
    f = (uint32_t)y;
  }
  // ((256 - w) x + w f + 128) >> 8 as one dot product of (x, f) with (256 - w, w).
  if (!(BPS == 1 && DIRECT)) xf = x | (f << 16);
  const uint32_t dot =
      __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, xf), __builtin_bit_cast(u16x2, pc.wp[p]), 128u, false);
  return RAW ? dot : dot >> 8;
}

// Four raw dot products (see one_sample) to one dword of samples: byte 1 of
// each, in order, by two byte permutes (selector byte 0x0c gives zero).
__device__ inline uint32_t pack_raw4(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3) {
  return __builtin_amdgcn_perm(r1, r0, 0x0c0c0501u) | __builtin_amdgcn_perm(r3, r2, 0x05010c0cu);
}

// Adds the workgroup's LDS histogram of camera `cam` (replicas summed) and
// its share of (n, S1, S2) - linear in the histogram for 8-bit samples, from
// the sample sums a1, a2 for 16-bit ones - to the camera's whole-frame
// statistics.
template <int C, int BPS>
__device__ inline void flush_whole(const Geo& g, const Bufs& b, int cam, ApplyLds& L, unsigned long long a1,
                                   unsigned long long a2) {
  const int tid = threadIdx.x;
  __syncthreads();
  uint32_t* gh = b.whole_hist + (int64_t)cam * kCS * kNB;
  uint32_t h[kCS];
#pragma unroll
  for (int c = 0; c < kCS; ++c) {
    uint32_t sum = 0;
    if (c < C) {
      if (kPack) {
        // Thread tid owns bin tid; the replica order is rotated per word so
        // that the lanes of a wave read distinct banks.
        const int wd = hist_word(c, (uint32_t)tid);
        const uint32_t sh = hist_shift((uint32_t)tid);
#pragma unroll 8
        for (int i = 0; i < kRep; ++i) sum += (L.hist[wd * kRep + ((i + wd) & (kRep - 1))] >> sh) & 0xffffu;
      } else {
#pragma unroll
        for (int r = 0; r < kRep; ++r) sum += L.hist[(c * kNB + tid) * kRep + r];
      }
    }
    h[c] = sum;
    if (sum) atomicAdd(&gh[c * kNB + tid], sum);
  }
  const unsigned long long x = (unsigned long long)tid;
  const unsigned long long h0 = h[0], h1 = h[1], h2 = h[2];
  block_sums(
      (BPS == 2) ? 3 : 3 * C,
      [=](int i) -> unsigned long long {
        const int c = i / 3, m = i - 3 * (i / 3);
        const unsigned long long hc = c == 0 ? h0 : (c == 1 ? h1 : h2);
        if (m == 0) return hc;
        if (BPS == 2) return m == 1 ? a1 : a2;
        return m == 1 ? hc * x : hc * x * x;
      },
      [&](int i, unsigned long long tot) {
        if (tot) atomicAdd((unsigned long long*)&b.whole_sums[(int64_t)cam * 9 + i], tot);
      },
      L.red);
}

// Segment ti of the context through the block's tables (8-bit samples:
// staged in LDS; 16-bit: the Q16 pairs).  WTAB: weights from the caller's
// table (true) or from their closed form (false); both give the same
// integers.  With statistics, `first` clears the LDS histogram (the first
// segment of its camera in this workgroup's run) and `last` adds it to the
// whole-frame statistics (the camera's last segment in the run); 16-bit
// samples, whose sums are kept in registers, and the packed histogram, whose
// counters are bounded per segment, do both on every segment.
template <int C, int BPS, bool WRITE, bool STATS, bool WTAB, class FP>
__device__ void apply_tile(const Geo& g, const FP& fp, const Bufs& b, int ti, ApplyLds& L, bool first,
                           bool last) {
  const bool clear = first || BPS == 2 || kPack;
  const bool flush = last || BPS == 2 || kPack;
  constexpr int NW = C * BPS;    // dwords per 4-pixel group
  constexpr int SPG = 4 * C;     // samples per group
  const int tid = threadIdx.x;
  const Tile t = uniform_tile(g.tiles[ti]);
  const DevCam cam = uniform_cam(g.cams[t.cam]);
  const int W = cam.width;
  const int half = cam.half;
  const int shift = cam.bit_depth - 8;
  const uint32_t maxv = (1u << cam.bit_depth) - 1u;
  const int pitch = (int)cam.pitch;

  // Stage the tables of both sides of the segment's block; clear the histogram.
  const int64_t u_left = unit_index(t.cam, 0, t.block, 0, g.n_blocks);
  const int64_t u_right = unit_index(t.cam, 1, t.block, 0, g.n_blocks);
  if (WRITE) {
    if (BPS == 1) {
      constexpr int DW = C * kNB / 4;   // dwords of one side's tables
      for (int i = tid; i < 2 * DW; i += kThreads) {
        const int s = i / DW;
        const int rem = i - s * DW;
        const uint32_t* src = reinterpret_cast<const uint32_t*>(b.lut8 + (s ? u_right : u_left) * kNB);
        reinterpret_cast<uint32_t*>(L.lut + s * kCS * kNB)[rem] = src[rem];
      }
    } else if (tid < 4) {
      L.q[tid] = b.q16[((tid >> 1) ? u_right : u_left) * 2 + (tid & 1)];
    }
  }
  if (STATS && clear) {
    for (int i = tid; i < kHistWords / kCS * C; i += kThreads) L.hist[i] = 0;
  }
  __syncthreads();

  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[t.cam], cam);
  __amdgpu_buffer_rsrc_t rout = rin;
  if (WRITE) rout = frame_rsrc(fp.out[t.cam], cam);
  const uint16_t* wrow = b.weights + (int64_t)t.cam * g.w_max;
  const int ngroups = (W + 3) >> 2;
  const int hrep = tid & (kRep - 1);
  unsigned long long a1 = 0, a2 = 0;

  for (int grp = tid; grp < ngroups; grp += kThreads) {
    const int col0 = grp * 4;
    const int npx = min(4, W - col0);
    PixConst pc;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int col = col0 + p;
      const int side = col < half ? 0 : 1;
      uint32_t w = 0;
      if (WRITE && p < npx) w = WTAB ? (uint32_t)wrow[col] : blend_weight(W, col);
      pc.wp[p] = (256u - w) | (w << 16);
      pc.lb[p] = side * kCS * kNB;
      if (BPS == 2 && WRITE) { pc.qa[p] = L.q[side * 2]; pc.qb[p] = L.q[side * 2 + 1]; }
    }
    const int cbyte = col0 * C * BPS;
    const Tile& ts = t;

    if (npx == 4) {
      for (int row = ts.r0; row < ts.r1; row += kUnroll) {
        uint32_t d[kUnroll][NW];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (row + u < ts.r1) load_group<NW>(rin, (row + u) * pitch + cbyte, d[u]);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (row + u < ts.r1) {
            uint32_t o[NW];
#pragma unroll
            for (int q = 0; q < NW; ++q) o[q] = 0;
#pragma unroll
            for (int i = 0; i < SPG; ++i) {
              const int p = i / C;
              const int c = i - p * C;
              uint32_t x;
              if (BPS == 1) x = (d[u][i >> 2] >> (8 * (i & 3))) & 0xffu;
              else x = (d[u][i >> 1] >> (16 * (i & 1))) & 0xffffu;
              const uint32_t y = one_sample<BPS, WRITE, STATS, false>(x, c, p, pc, L, hrep, shift, maxv, a1, a2);
              if (WRITE) {
                if (BPS == 1) o[i >> 2] |= y << (8 * (i & 3));
                else o[i >> 1] |= y << (16 * (i & 1));
              }
            }
            if (WRITE) store_group<NW>(rout, (row + u) * pitch + cbyte, o);
          }
        }
      }
    } else {
      // Ragged end of the row: sample by sample, touching only the row's bytes.
      for (int row = ts.r0; row < ts.r1; ++row) {
        const int off = row * pitch + cbyte;
#pragma unroll
        for (int i = 0; i < SPG; ++i) {
          const int p = i / C;
          const int c = i - p * C;
          if (p < npx) {
            uint32_t x;
            if (BPS == 1) x = __builtin_amdgcn_raw_buffer_load_b8(rin, off + i, 0, 0);
            else x = __builtin_amdgcn_raw_buffer_load_b16(rin, off + 2 * i, 0, 0);
            const uint32_t y = one_sample<BPS, WRITE, STATS, false>(x, c, p, pc, L, hrep, shift, maxv, a1, a2);
            if (WRITE) {
              if (BPS == 1) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)y, rout, off + i, 0, 0);
              else __builtin_amdgcn_raw_buffer_store_b16((uint16_t)y, rout, off + 2 * i, 0, 0);
            }
          }
        }
      }
    }
  }

  if (STATS && flush) flush_whole<C, BPS>(g, b, t.cam, L, a1, a2);
}

// Row-wise blend of adjacent blocks' maps (section 5's convex combinations of
// the maps of adjacent blocks; every block holds at least one row): with
// doubled block centres C_j = r0_j + r1_j - 1, row r of block j blends j with
// its neighbour on r's side of the centre (alone before the first and from
// the last centre on), weight v of the second block = round_half_up(256
// (2r - C_a) / (C_b - C_a)); each Q16 parameter of the row is
// floor(((256 - v) P_a + v P_b + 128) / 256).
__device__ inline int block_centre2(int j, int H, int nb) {
  return (int)((int64_t)j * H / nb) + (int)((int64_t)(j + 1) * H / nb) - 1;
}

__device__ inline void vblend_row(int H, int nb, int r, int& a, int& b, int& v) {
  const int j = (int)(((int64_t)(r + 1) * nb - 1) / H);
  const int lo = 2 * r < block_centre2(j, H, nb) ? j - 1 : j;
  if (lo < 0 || lo + 1 >= nb) {
    a = b = j;
    v = 0;
    return;
  }
  const int ca = block_centre2(lo, H, nb), cb = block_centre2(lo + 1, H, nb);
  a = lo;
  b = lo + 1;
  v = ((2 * r - ca) * 512 + (cb - ca)) / (2 * (cb - ca));
}

__device__ inline int64_t blend_q16(int64_t pa, int64_t pb, int v) {
  return ((256 - v) * pa + v * pb + 128) >> 8;
}

// Apply (and statistics) of segment ti with the maps blended row by row.
// Each row's blended Q16 pairs of both sides are computed once per row
// (uniform over the workgroup) and every sample is evaluated from its side's
// pair in 64-bit integers, 8-bit and 16-bit samples alike.  Same histogram
// and flush as apply_tile.
template <int C, int BPS, bool WRITE, bool STATS, bool WTAB, class FP>
__device__ void apply_tile_vblend(const Geo& g, const FP& fp, const Bufs& b, int ti, ApplyLds& L,
                                  bool first, bool last) {
  const bool clear = first || BPS == 2 || kPack;
  const bool flush = last || BPS == 2 || kPack;
  constexpr int SPG = 4 * C;     // samples per group
  const int tid = threadIdx.x;
  const Tile t = uniform_tile(g.tiles[ti]);
  const DevCam cam = uniform_cam(g.cams[t.cam]);
  const int W = cam.width, H = cam.height, half = cam.half, nb = g.n_blocks;
  const int shift = cam.bit_depth - 8;
  const uint32_t maxv = (1u << cam.bit_depth) - 1u;
  const int pitch = (int)cam.pitch;
  if (STATS && clear) {
    for (int i = tid; i < kHistWords / kCS * C; i += kThreads) L.hist[i] = 0;
  }
  __syncthreads();
  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[t.cam], cam);
  __amdgpu_buffer_rsrc_t rout = rin;
  if (WRITE) rout = frame_rsrc(fp.out[t.cam], cam);
  const uint16_t* wrow = b.weights + (int64_t)t.cam * g.w_max;
  const int hrep = tid & (kRep - 1);
  unsigned long long a1 = 0, a2 = 0;
  const int ngroups = (W + 3) >> 2;
  for (int grp = tid; grp < ngroups; grp += kThreads) {
    const int col0 = grp * 4, npx = min(4, W - col0);
    uint32_t wp[4];
    bool right[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int col = col0 + p;
      uint32_t w = 0;
      if (WRITE && p < npx) w = WTAB ? (uint32_t)wrow[col] : blend_weight(W, col);
      wp[p] = (256u - w) | (w << 16);
      right[p] = col >= half;
    }
    for (int row = t.r0; row < t.r1; ++row) {
      int ja, jb, v;
      vblend_row(H, nb, row, ja, jb, v);
      int64_t A[2][kCS], Bq[2][kCS];
      if (WRITE) {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const int64_t ua = unit_index(t.cam, sd, ja, c, nb), ub = unit_index(t.cam, sd, jb, c, nb);
            A[sd][c] = blend_q16(uniform(b.q16[ua * 2]), uniform(b.q16[ub * 2]), v);
            Bq[sd][c] = blend_q16(uniform(b.q16[ua * 2 + 1]), uniform(b.q16[ub * 2 + 1]), v);
          }
      }
      const int off = row * pitch + col0 * C * BPS;
#pragma unroll
      for (int i = 0; i < SPG; ++i) {
        const int p = i / C, c = i - p * C;
        if (p < npx) {
          const uint32_t x = BPS == 1 ? __builtin_amdgcn_raw_buffer_load_b8(rin, off + i, 0, 0)
                                      : __builtin_amdgcn_raw_buffer_load_b16(rin, off + 2 * i, 0, 0);
          if (STATS) {
            uint32_t bin = x;
            if (BPS == 2) { bin = x >> shift; bin = bin > 255u ? 255u : bin; }
            __hip_atomic_fetch_add(&L.hist[hist_word(c, bin) * kRep + hrep], 1u << hist_shift(bin),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (BPS == 2) { a1 += x; a2 += (unsigned long long)x * x; }
          }
          if (WRITE) {
            const int sd = right[p] ? 1 : 0;
            int64_t y = (A[sd][c] * (int64_t)x + Bq[sd][c] + 32768) >> 16;
            y = y < 0 ? 0 : (y > (int64_t)maxv ? (int64_t)maxv : y);
            const uint32_t xf = x | ((uint32_t)y << 16);
            const uint32_t o = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, xf),
                                                      __builtin_bit_cast(u16x2, wp[p]), 128u, false) >> 8;
            if (BPS == 1) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)o, rout, off + i, 0, 0);
            else __builtin_amdgcn_raw_buffer_store_b16((uint16_t)o, rout, off + 2 * i, 0, 0);
          }
        }
      }
    }
  }
  if (STATS && flush) flush_whole<C, BPS>(g, b, t.cam, L, a1, a2);
}

// Direct-map constants of this many blocks fit in the LDS table area.
constexpr int kRunBlocks = (int)(sizeof(ApplyLds::lut) / (2 * kCS * 2 * sizeof(int32_t)));

// Apply with statistics over segments [ti, te) of one 8-bit camera: their
// rows are consecutive and every block among them has direct maps (at most
// kRunBlocks blocks).  One row loop covers all the segments: the blocks'
// constants are staged in LDS, and at a block's first row each thread
// re-selects its pixels' constants (by side) from them, so a block boundary
// costs no memory latency and no partly filled unroll step.  Same results as
// apply_tile.
template <int C, bool WTAB, class FP>
__device__ void apply_run_direct(const Geo& g, const FP& fp, const Bufs& b, int ti, int te, ApplyLds& L,
                                 bool first, bool last) {
  constexpr int NW = C;          // dwords per 4-pixel group
  const int tid = threadIdx.x;
  const Tile t0 = uniform_tile(g.tiles[ti]);
  const int R0 = t0.r0, R1 = uniform(g.tiles[te - 1].r1);
  const int j0 = t0.block, j1 = uniform(g.tiles[te - 1].block);
  const DevCam cam = uniform_cam(g.cams[t0.cam]);
  const int W = cam.width, half = cam.half, H = cam.height, nb = g.n_blocks;
  const int pitch = (int)cam.pitch;

  // [block - j0][side][channel][a, c]
  int32_t* cst = reinterpret_cast<int32_t*>(L.lut);
  for (int i = tid; i < (j1 - j0 + 1) * 2 * kCS; i += kThreads) {
    const int jj = i / (2 * kCS), sd = (i / kCS) & 1, c = i % kCS;
    const int64_t u = unit_index(t0.cam, sd, j0 + jj, c, nb);
    cst[i * 2] = (int32_t)b.q16[u * 2];
    cst[i * 2 + 1] = (int32_t)(b.q16[u * 2 + 1] + 32768);
  }
  if (first || kPack)
    for (int i = tid; i < kHistWords / kCS * C; i += kThreads) L.hist[i] = 0;
  __syncthreads();

  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[t0.cam], cam);
  const __amdgpu_buffer_rsrc_t rout = frame_rsrc(fp.out[t0.cam], cam);
  const uint16_t* wrow = b.weights + (int64_t)t0.cam * g.w_max;
  const int hrep = tid & (kRep - 1);
  const int ngroups = (W + 3) >> 2;
  unsigned long long a1 = 0, a2 = 0;

  for (int grp = tid; grp < ngroups; grp += kThreads) {
    const int col0 = grp * 4;
    const int npx = min(4, W - col0);
    PixConst pc;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint32_t w = p < npx ? (WTAB ? (uint32_t)wrow[col0 + p] : blend_weight(W, col0 + p)) : 0u;
      pc.wp[p] = (256u - w) | (w << 16);
    }
    int jb = j0;
    int rb = min(R1, (int)((int64_t)(jb + 1) * H / nb));   // first row of the next block
    auto select = [&]() {
      int32_t A[2][kCS], Cc[2][kCS];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int c = 0; c < kCS; ++c) {
          const int i = (((jb - j0) * 2 + sd) * kCS + c) * 2;
          A[sd][c] = uniform(cst[i]);
          Cc[sd][c] = uniform(cst[i + 1]);
        }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const bool right = col0 + p >= half;
#pragma unroll
        for (int c = 0; c < kCS; ++c) {
          pc.da[p][c] = right ? A[1][c] : A[0][c];
          pc.dc[p][c] = right ? Cc[1][c] : Cc[0][c];
        }
      }
    };
    select();
    // Row r starts block jb + 1 when r == rb.  Blocks hold no rows when
    // H < NB, so several block starts can fall on one row: step over every
    // empty block to the one that holds r (uniform over the wave).
    auto next_block = [&](int r) {
      if (r != rb) return;
      while (r == rb && jb < j1) {
        ++jb;
        rb = min(R1, (int)((int64_t)(jb + 1) * H / nb));
      }
      select();
    };
    const int cbyte = col0 * C;

    if (npx == 4) {
      for (int row = R0; row < R1; row += kUnroll) {
        uint32_t d[kUnroll][NW];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (row + u < R1) load_group<NW>(rin, (row + u) * pitch + cbyte, d[u]);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (row + u < R1) {
            next_block(row + u);
            uint32_t r[4 * C], o[NW];
#pragma unroll
            for (int i = 0; i < 4 * C; ++i) {
              const int p = i / C, c = i - (i / C) * C;
              const uint32_t x = (d[u][i >> 2] >> (8 * (i & 3))) & 0xffu;
              r[i] = one_sample<1, true, true, true, true>(x, c, p, pc, L, hrep, 0, 255u, a1, a2);
            }
#pragma unroll
            for (int q = 0; q < NW; ++q) o[q] = pack_raw4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
            store_group<NW>(rout, (row + u) * pitch + cbyte, o);
          }
        }
      }
    } else {
      // Ragged end of the row: sample by sample, touching only the row's bytes.
      for (int row = R0; row < R1; ++row) {
        next_block(row);
        const int off = row * pitch + cbyte;
#pragma unroll
        for (int i = 0; i < 4 * C; ++i) {
          const int p = i / C, c = i - (i / C) * C;
          if (p < npx) {
            const uint32_t x = __builtin_amdgcn_raw_buffer_load_b8(rin, off + i, 0, 0);
            const uint32_t y = one_sample<1, true, true, true>(x, c, p, pc, L, hrep, 0, 255u, a1, a2);
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)y, rout, off + i, 0, 0);
          }
        }
      }
    }
  }
  if (last || kPack) flush_whole<C, 1>(g, b, t0.cam, L, 0ull, 0ull);
}

// Whether every row map blended from blocks [js, je] of camera k can be
// evaluated directly (uniform): a blended pair lies between its two blocks'
// pairs (floor of a convex combination plus one half), so |A| < 2^23 and
// 255 max|A| + max|Bq + 2^15| < 2^31 over the blocks bound every row's
// A x + Bq + 2^15 inside int32.
__device__ inline bool vblend_direct_ok(const Geo& g, const Bufs& b, int k, int js, int je) {
  int64_t ma = 0, mc = 0;
  for (int j = js; j <= je; ++j)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int c = 0; c < kCS; ++c) {
        const int64_t u = unit_index(k, sd, j, c, g.n_blocks);
        const int64_t A = uniform(b.q16[u * 2]), C = uniform(b.q16[u * 2 + 1]) + 32768;
        ma = max(ma, A < 0 ? -A : A);
        mc = max(mc, C < 0 ? -C : C);
      }
  return ma < (1 << 23) && 255 * ma + mc <= (int64_t)INT32_MAX;
}

// Rows whose blended direct constants fit the LDS table area.
constexpr int kVblendRows = (int)(sizeof(ApplyLds::lut) / (2 * kCS * 2 * sizeof(int32_t)));

// Apply of segments [ti, te) of one 8-bit camera with the maps blended row
// by row (apply_tile_vblend's results), kVblendRows rows at a time: one
// thread per row blends the row's two blocks' Q16 pairs of both sides into
// direct constants in LDS, then every thread takes its pixels' constants of
// each row from there and the samples follow the direct path of
// apply_run_direct.
template <int C, bool STATS, bool WTAB, class FP>
__device__ void apply_run_vblend(const Geo& g, const FP& fp, const Bufs& b, int ti, int te, ApplyLds& L,
                                 bool first, bool last) {
  constexpr int NW = C;
  const int tid = threadIdx.x;
  const Tile t0 = uniform_tile(g.tiles[ti]);
  const int R0 = t0.r0, R1 = uniform(g.tiles[te - 1].r1);
  const DevCam cam = uniform_cam(g.cams[t0.cam]);
  const int W = cam.width, half = cam.half, H = cam.height, nb = g.n_blocks;
  const int pitch = (int)cam.pitch;
  int32_t* rc = reinterpret_cast<int32_t*>(L.lut);   // [row - chunk start][side][channel][A, Bq + 2^15]
  if (STATS && (first || kPack))
    for (int i = tid; i < kHistWords / kCS * C; i += kThreads) L.hist[i] = 0;
  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[t0.cam], cam);
  const __amdgpu_buffer_rsrc_t rout = frame_rsrc(fp.out[t0.cam], cam);
  const uint16_t* wrow = b.weights + (int64_t)t0.cam * g.w_max;
  const int hrep = tid & (kRep - 1);
  const int ngroups = (W + 3) >> 2;
  unsigned long long a1 = 0, a2 = 0;

  for (int c0 = R0; c0 < R1; c0 += kVblendRows) {
    const int c1 = min(c0 + kVblendRows, R1);
    __syncthreads();   // the previous chunk's rows are done with the table
    if (tid < c1 - c0) {
      int ja, jb, v;
      vblend_row(H, nb, c0 + tid, ja, jb, v);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int c = 0; c < kCS; ++c) {
          const int64_t ua = unit_index(t0.cam, sd, ja, c, nb), ub = unit_index(t0.cam, sd, jb, c, nb);
          const int i = ((tid * 2 + sd) * kCS + c) * 2;
          rc[i] = (int32_t)blend_q16(b.q16[ua * 2], b.q16[ub * 2], v);
          rc[i + 1] = (int32_t)(blend_q16(b.q16[ua * 2 + 1], b.q16[ub * 2 + 1], v) + 32768);
        }
    }
    __syncthreads();
    for (int grp = tid; grp < ngroups; grp += kThreads) {
      const int col0 = grp * 4;
      const int npx = min(4, W - col0);
      PixConst pc;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const uint32_t w = p < npx ? (WTAB ? (uint32_t)wrow[col0 + p] : blend_weight(W, col0 + p)) : 0u;
        pc.wp[p] = (256u - w) | (w << 16);
      }
      // A group on one side of the centre takes one side's constants (three
      // 8-byte LDS reads per row); only the group across the centre, if
      // any, selects per pixel.
      const bool one_side = (col0 >= half) == (col0 + 3 >= half);
      const int side0 = col0 >= half ? kCS * 2 : 0;
      auto select_row = [&](int r) {
        const int base = (r - c0) * 2 * kCS * 2;
        if (one_side) {
          const int2* q = reinterpret_cast<const int2*>(rc + base + side0);
#pragma unroll
          for (int c = 0; c < kCS; ++c) {
            const int2 v = q[c];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              pc.da[p][c] = v.x;
              pc.dc[p][c] = v.y;
            }
          }
          return;
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int sb = base + (col0 + p >= half ? kCS * 2 : 0);
#pragma unroll
          for (int c = 0; c < kCS; ++c) {
            pc.da[p][c] = rc[sb + c * 2];
            pc.dc[p][c] = rc[sb + c * 2 + 1];
          }
        }
      };
      const int cbyte = col0 * C;
      if (npx == 4) {
        for (int row = c0; row < c1; row += kUnroll) {
          uint32_t d[kUnroll][NW];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
            if (row + u < c1) load_group<NW>(rin, (row + u) * pitch + cbyte, d[u]);
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            if (row + u < c1) {
              select_row(row + u);
              uint32_t r[4 * C], o[NW];
#pragma unroll
              for (int i = 0; i < 4 * C; ++i) {
                const int p = i / C, c = i - (i / C) * C;
                const uint32_t x = (d[u][i >> 2] >> (8 * (i & 3))) & 0xffu;
                r[i] = one_sample<1, true, STATS, true, true>(x, c, p, pc, L, hrep, 0, 255u, a1, a2);
              }
#pragma unroll
              for (int q = 0; q < NW; ++q) o[q] = pack_raw4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
              store_group<NW>(rout, (row + u) * pitch + cbyte, o);
            }
          }
        }
      } else {
        // Ragged end of the row: sample by sample, touching only the row's bytes.
        for (int row = c0; row < c1; ++row) {
          select_row(row);
          const int off = row * pitch + cbyte;
#pragma unroll
          for (int i = 0; i < 4 * C; ++i) {
            const int p = i / C, c = i - (i / C) * C;
            if (p < npx) {
              const uint32_t x = __builtin_amdgcn_raw_buffer_load_b8(rin, off + i, 0, 0);
              const uint32_t y = one_sample<1, true, STATS, true>(x, c, p, pc, L, hrep, 0, 255u, a1, a2);
              __builtin_amdgcn_raw_buffer_store_b8((uint8_t)y, rout, off + i, 0, 0);
            }
          }
        }
      }
    }
  }
  if (STATS && (last || kPack)) flush_whole<C, 1>(g, b, t0.cam, L, 0ull, 0ull);
}

// Whether the six 8-bit maps of segment ti can be evaluated directly (uniform).
__device__ inline bool tile_direct(const Geo& g, const Bufs& b, int ti) {
  const Tile t = uniform_tile(g.tiles[ti]);
  bool ok = true;
#pragma unroll
  for (int sd = 0; sd < 2; ++sd)
#pragma unroll
    for (int c = 0; c < kCS; ++c) {
      const int64_t u = unit_index(t.cam, sd, t.block, c, g.n_blocks);
      ok = ok && direct_ok(uniform(b.q16[u * 2]), uniform(b.q16[u * 2 + 1]));
    }
  return ok;
}

// The segments from ti on, up to se, that one call takes: with the direct
// maps (8-bit samples, apply with statistics, every segment's maps direct),
// the camera's consecutive segments (apply_run_direct); otherwise one
// (apply_tile).  Returns the end of the segments taken; `last` is set when
// they end the camera's run in this workgroup.
template <bool WRITE, bool STATS, bool WTAB, bool VBLEND = false, class FP = FramePtrs>
__device__ inline int apply_tile_dispatch(const Geo& g, const FP& fp, const Bufs& b, int ti, int se,
                                          ApplyLds& L, bool first) {
  const int k = uniform(g.tiles[ti].cam);
  const DevCam cam = uniform_cam(g.cams[k]);
  int te = ti + 1;
  if constexpr (VBLEND) {
    const int j0 = uniform(g.tiles[ti].block);
    if (cam.bps == 1 && WRITE && RC_APPLY_DIRECT &&
        vblend_direct_ok(g, b, k, j0 > 0 ? j0 - 1 : 0, min(j0 + 1, g.n_blocks - 1))) {
      // A camera's consecutive segments whose blocks and neighbours fit the
      // staging area and evaluate directly.
      const int cap = max_tile_rows(cam.width), r0 = uniform(g.tiles[ti].r0);
      while (te < se && uniform(g.tiles[te].cam) == k && uniform(g.tiles[te].r1) - r0 <= cap) {
        const int jt = uniform(g.tiles[te].block);
        if (!vblend_direct_ok(g, b, k, jt, min(jt + 1, g.n_blocks - 1))) break;
        ++te;
      }
      const bool lastr = te == se || uniform(g.tiles[te].cam) != k;
      if (cam.channels == 3) apply_run_vblend<3, STATS, WTAB>(g, fp, b, ti, te, L, first, lastr);
      else apply_run_vblend<1, STATS, WTAB>(g, fp, b, ti, te, L, first, lastr);
      return te;
    }
    const bool lastv = te == se || uniform(g.tiles[te].cam) != k;
    if (cam.bps == 2) apply_tile_vblend<1, 2, WRITE, STATS, WTAB>(g, fp, b, ti, L, first, lastv);
    else if (cam.channels == 3) apply_tile_vblend<3, 1, WRITE, STATS, WTAB>(g, fp, b, ti, L, first, lastv);
    else apply_tile_vblend<1, 1, WRITE, STATS, WTAB>(g, fp, b, ti, L, first, lastv);
    return te;
  }
  const bool direct = cam.bps == 1 && WRITE && STATS && RC_APPLY_DIRECT && tile_direct(g, b, ti);
  const int j0 = uniform(g.tiles[ti].block);
  // Packed counters bound the rows between flushes.
  const int cap = max_tile_rows(cam.width), r0 = uniform(g.tiles[ti].r0);
  if (direct)
    while (te < se && uniform(g.tiles[te].cam) == k && uniform(g.tiles[te].block) - j0 < kRunBlocks &&
           uniform(g.tiles[te].r1) - r0 <= cap && tile_direct(g, b, te))
      ++te;
  const bool last = te == se || uniform(g.tiles[te].cam) != k;
  if (cam.bps == 2) apply_tile<1, 2, WRITE, STATS, WTAB>(g, fp, b, ti, L, first, last);
  else if (direct) {
    // Measured on MI355X: faster than the LDS tables when the pass also
    // builds the histogram (the LDS is then busy with its atomics), slower
    // for the apply alone.
    if (cam.channels == 3) apply_run_direct<3, WTAB>(g, fp, b, ti, te, L, first, last);
    else apply_run_direct<1, WTAB>(g, fp, b, ti, te, L, first, last);
  } else if (cam.channels == 3) apply_tile<3, 1, WRITE, STATS, WTAB>(g, fp, b, ti, L, first, last);
  else apply_tile<1, 1, WRITE, STATS, WTAB>(g, fp, b, ti, L, first, last);
  return te;
}

}  // namespace rc
