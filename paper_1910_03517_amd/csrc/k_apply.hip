// Apply pass of section 3.1: every sample is blended between the identity and
// its side's affine map, with the Q8 weight of its column, in exact integer
// arithmetic; optionally fused with the whole-frame statistics of the input.
//
// Work split: one workgroup per tile (camera, block, row range).  A thread
// owns groups of 4 consecutive pixels of the row (12 bytes for RGB8, 4 for
// gray8, 8 for gray16) and walks down the tile's rows, so that the weights and
// table bases of its pixels stay in registers.  The tile's tables sit in LDS;
// the histogram is privatised in LDS and merged once per tile.  Frames are
// accessed through buffer resources sized to the frame, so the hardware range
// check covers every access.
#include "rt_internal.h"

namespace rc {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));

constexpr int kApplyThreads = 256;
template <int NW>
__device__ inline void load_group(__amdgpu_buffer_rsrc_t r, int off, uint32_t (&d)[NW]) {
  if constexpr (NW == 3) {
    u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
    d[0] = v.x; d[1] = v.y; d[2] = v.z;
  } else if constexpr (NW == 2) {
    u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    d[0] = v.x; d[1] = v.y;
  } else {
    d[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  }
}

template <int NW>
__device__ inline void store_group(__amdgpu_buffer_rsrc_t r, int off, const uint32_t (&d)[NW]) {
  if constexpr (NW == 3) {
    u32x3 v = {d[0], d[1], d[2]};
    __builtin_amdgcn_raw_buffer_store_b96(v, r, off, 0, 0);
  } else if constexpr (NW == 2) {
    u32x2 v = {d[0], d[1]};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(d[0], r, off, 0, 0);
  }
}

// The blend of one sample: y = ((256 - w) x + w f + 128) >> 8.
__device__ inline uint32_t blend(uint32_t x, uint32_t f, uint32_t w) {
  return ((256u - w) * x + w * f + 128u) >> 8;
}

template <int C, int BPS, bool WRITE, bool STATS>
__device__ void apply_tile(const Geo& g, const FramePtrs& fp, const Bufs& b, const Tile& t,
                           uint8_t* s_lut, int64_t* s_q, uint32_t* s_hist, unsigned long long* s_acc) {
  constexpr int NW = C * BPS;           // dwords per 4-pixel group
  constexpr int SPG = 4 * C;            // samples per group
  const int tid = threadIdx.x;
  const DevCam cam = g.cams[t.cam];
  const int W = cam.width;
  const int half = cam.half;
  const int shift = cam.bit_depth - 8;
  const uint32_t maxv = (1u << cam.bit_depth) - 1u;

  // Stage the tile's tables (both sides of block t.block) and clear the histogram.
  const int64_t u_left = unit_index(t.cam, 0, t.block, 0, g.n_blocks);
  const int64_t u_right = unit_index(t.cam, 1, t.block, 0, g.n_blocks);
  if (WRITE) {
    if (BPS == 1) {
      for (int i = tid; i < 2 * C * kNB; i += kApplyThreads) {
        const int s = i / (C * kNB);
        const int rem = i - s * C * kNB;
        s_lut[s * kCS * kNB + rem] = b.lut8[(s ? u_right : u_left) * kNB + rem];
      }
    } else if (tid < 4) {
      const int s = tid >> 1;
      s_q[tid] = b.q16[(s ? u_right : u_left) * 2 + (tid & 1)];
    }
  }
  if (STATS) {
    for (int i = tid; i < C * kNB; i += kApplyThreads) s_hist[i] = 0;
    if (BPS == 2 && tid < 2) s_acc[tid] = 0;
  }
  __syncthreads();

  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[t.cam], cam);
  __amdgpu_buffer_rsrc_t rout = rin;
  if (WRITE) rout = frame_rsrc(fp.out[t.cam], cam);
  const uint16_t* wrow = b.weights + (int64_t)t.cam * g.w_max;
  const int ngroups = (W + 3) >> 2;
  unsigned long long acc1 = 0, acc2 = 0;

  for (int grp = tid; grp < ngroups; grp += kApplyThreads) {
    const int col0 = grp * 4;
    const int npx = min(4, W - col0);
    uint32_t wv[4];
    int lb[4];
    int64_t qa[4], qb[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int col = col0 + p;
      const int side = col < half ? 0 : 1;
      const uint32_t wtab = WRITE ? (uint32_t)wrow[col < W ? col : W - 1] : 0u;
      wv[p] = p < npx ? wtab : 0u;
      lb[p] = side * kCS * kNB;
      if (BPS == 2 && WRITE) { qa[p] = s_q[side * 2]; qb[p] = s_q[side * 2 + 1]; }
    }
    const int cbyte = col0 * C * BPS;

    if (npx == 4) {
      for (int row = t.r0; row < t.r1; ++row) {
        const int off = (int)((int64_t)row * cam.pitch) + cbyte;
        uint32_t d[NW];
        load_group<NW>(rin, off, d);
        uint32_t o[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) o[q] = 0;
#pragma unroll
        for (int i = 0; i < SPG; ++i) {
          const int p = i / C;
          const int c = i - p * C;
          uint32_t x;
          if (BPS == 1) x = (d[i >> 2] >> (8 * (i & 3))) & 0xffu;
          else x = (d[i >> 1] >> (16 * (i & 1))) & 0xffffu;
          if (STATS) {
            uint32_t bin = x;
            if (BPS == 2) { bin = x >> shift; bin = bin > 255u ? 255u : bin; }
            atomicAdd(&s_hist[c * kNB + bin], 1u);
            if (BPS == 2) { acc1 += x; acc2 += (unsigned long long)x * x; }
          }
          if (WRITE) {
            uint32_t f;
            if (BPS == 1) {
              f = s_lut[lb[p] + c * kNB + x];
            } else {
              int64_t y = (qa[p] * (int64_t)x + qb[p] + 32768) >> 16;
              y = y < 0 ? 0 : (y > (int64_t)maxv ? (int64_t)maxv : y);
              f = (uint32_t)y;
            }
            const uint32_t yv = blend(x, f, wv[p]);
            if (BPS == 1) o[i >> 2] |= yv << (8 * (i & 3));
            else o[i >> 1] |= yv << (16 * (i & 1));
          }
        }
        if (WRITE) store_group<NW>(rout, off, o);
      }
    } else {
      // Ragged end of the row: sample by sample, touching only the row's bytes.
      for (int row = t.r0; row < t.r1; ++row) {
        const int off = (int)((int64_t)row * cam.pitch) + cbyte;
        for (int i = 0; i < npx * C; ++i) {
          const int p = i / C;
          const int c = i - p * C;
          uint32_t x;
          if (BPS == 1) x = __builtin_amdgcn_raw_buffer_load_b8(rin, off + i, 0, 0);
          else x = __builtin_amdgcn_raw_buffer_load_b16(rin, off + 2 * i, 0, 0);
          if (STATS) {
            uint32_t bin = x;
            if (BPS == 2) { bin = x >> shift; bin = bin > 255u ? 255u : bin; }
            atomicAdd(&s_hist[c * kNB + bin], 1u);
            if (BPS == 2) { acc1 += x; acc2 += (unsigned long long)x * x; }
          }
          if (WRITE) {
            uint32_t f;
            if (BPS == 1) {
              f = s_lut[lb[p] + c * kNB + x];
            } else {
              int64_t y = (qa[p] * (int64_t)x + qb[p] + 32768) >> 16;
              y = y < 0 ? 0 : (y > (int64_t)maxv ? (int64_t)maxv : y);
              f = (uint32_t)y;
            }
            const uint32_t yv = blend(x, f, wv[p]);
            if (BPS == 1) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)yv, rout, off + i, 0, 0);
            else __builtin_amdgcn_raw_buffer_store_b16((uint16_t)yv, rout, off + 2 * i, 0, 0);
          }
        }
      }
    }
  }

  if (STATS) {
    if (BPS == 2) {
      if (acc1) atomicAdd(&s_acc[0], acc1);
      if (acc2) atomicAdd(&s_acc[1], acc2);
    }
    __syncthreads();
    uint32_t* gh = b.whole_hist + (int64_t)t.cam * kCS * kNB;
    for (int i = tid; i < C * kNB; i += kApplyThreads) {
      const uint32_t v = s_hist[i];
      if (v) atomicAdd(&gh[i], v);
    }
    if (BPS == 2 && tid == 0) {
      uint64_t* gs = b.whole_sums + (int64_t)t.cam * kCS * 3;
      atomicAdd((unsigned long long*)&gs[0], (unsigned long long)(t.r1 - t.r0) * (unsigned long long)W);
      atomicAdd((unsigned long long*)&gs[1], s_acc[0]);
      atomicAdd((unsigned long long*)&gs[2], s_acc[1]);
    }
  }
}

template <bool WRITE, bool STATS>
__global__ __launch_bounds__(kApplyThreads) void k_apply(Geo g, FramePtrs fp, Bufs b) {
  __shared__ uint8_t s_lut[2 * kCS * kNB];
  __shared__ int64_t s_q[4];
  __shared__ uint32_t s_hist[kCS * kNB];
  __shared__ unsigned long long s_acc[2];
  const Tile t = g.tiles[blockIdx.x];
  const DevCam& cam = g.cams[t.cam];
  if (cam.bps == 2) apply_tile<1, 2, WRITE, STATS>(g, fp, b, t, s_lut, s_q, s_hist, s_acc);
  else if (cam.channels == 3) apply_tile<3, 1, WRITE, STATS>(g, fp, b, t, s_lut, s_q, s_hist, s_acc);
  else apply_tile<1, 1, WRITE, STATS>(g, fp, b, t, s_lut, s_q, s_hist, s_acc);
}

hipError_t launch_apply(const Geo& g, const FramePtrs& fp, const Bufs& b, bool with_stats, hipStream_t st) {
  if (with_stats) hipLaunchKernelGGL((k_apply<true, true>), dim3(g.n_tiles), dim3(kApplyThreads), 0, st, g, fp, b);
  else hipLaunchKernelGGL((k_apply<true, false>), dim3(g.n_tiles), dim3(kApplyThreads), 0, st, g, fp, b);
  return hipGetLastError();
}

hipError_t launch_whole_stats(const Geo& g, const FramePtrs& fp, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL((k_apply<false, true>), dim3(g.n_tiles), dim3(kApplyThreads), 0, st, g, fp, b);
  return hipGetLastError();
}

}  // namespace rc
