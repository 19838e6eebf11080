// Internal declarations of the ringcorr HIP library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ringcorr.h"

namespace rc {

constexpr int kCS = RT_CSLOTS;   // channel slots
constexpr int kNB = RT_NBINS;    // histogram bins
constexpr int kThreads = 256;    // threads of every workgroup
constexpr int kMlpIn = RT_MLP_IN, kMlpHid = RT_MLP_HID, kMlpOut = RT_MLP_OUT;

// Whole-frame histogram of the apply pass: replicas, and whether two bins
// share a word as 16-bit halves (1: bins 2i, 2i + 1; 2: bins i, i + 128).
#ifndef RC_APPLY_PACK
#define RC_APPLY_PACK 0
#endif
#ifndef RC_APPLY_REP
#define RC_APPLY_REP (RC_APPLY_PACK ? 16 : 8)
#endif
static_assert(kThreads % RC_APPLY_REP == 0 && (RC_APPLY_REP & (RC_APPLY_REP - 1)) == 0, "replicas");

// Most rows one apply tile of a camera of this width may hold so that no
// packed 16-bit counter overflows: replica r is updated by the threads with
// tid % REP == r, which own the 4-pixel column groups g with g % REP == r, so
// a tile adds at most 4 * ceil(groups / REP) * rows to one counter.
__host__ __device__ inline int max_tile_rows(int width) {
  if (!RC_APPLY_PACK) return 1 << 30;
  const int groups = (width + 3) / 4;
  const int per_rep = (groups + RC_APPLY_REP - 1) / RC_APPLY_REP;
  return 65535 / (4 * per_rep);
}

// Per-camera geometry as the kernels see it (uploaded once per context).
struct DevCam {
  int32_t width, height, channels, bit_depth;
  int32_t bps;           // bytes per sample: 1 or 2
  int32_t band;          // band width clamped to floor(W/2)
  int32_t half;          // floor(W/2)
  int32_t row_bytes;     // width * channels * bps
  int32_t face_cam[2];   // camera facing side s, -1 if none (open chain end)
  int32_t face_side[2];
  int32_t tile_begin;    // this camera's tiles are [tile_begin, tile_end)
  int32_t tile_end;
  int64_t pitch;         // bytes between rows
};

// One segment of the apply pass: rows [r0, r1) of block `block` of camera
// `cam`.  Each apply workgroup takes a contiguous run of segments.
struct Tile {
  int32_t cam, block, r0, r1;
};

// Frame pointers of one launch, passed by value as a kernel argument.
struct FramePtrs {
  const uint8_t* in[RT_MAX_CAMS];
  uint8_t* out[RT_MAX_CAMS];
};

// Several frame-sets of one rig in one apply launch: set f takes workgroups
// [f * n_wg, (f + 1) * n_wg), its frames at index [f][k] and its own tables,
// weights and whole-frame buffers (the pipeline's slots).
// Sized so that the kernel argument stays near the single-set one.
constexpr int kSetsMax = 4;    // frame-sets per launch
constexpr int kSetCams = 16;   // cameras per frame-set
struct SetFrames {
  const uint8_t* in[kSetCams];
  uint8_t* out[kSetCams];
};
struct SetBufs {
  uint32_t* whole_hist;
  uint64_t* whole_sums;
  uint8_t* lut8;
  int64_t* q16;
  uint16_t* weights;
};
struct SetPtrs {
  SetFrames f[kSetsMax];
  SetBufs b[kSetsMax];
  int32_t n_sets;
};

// Caller buffers (device pointers) of one launch.
struct Bufs {
  uint32_t* band_hist;
  uint64_t* band_sums;
  uint32_t* whole_hist;
  uint64_t* whole_sums;
  double* params;
  uint8_t* valid;
  uint8_t* lut8;
  int64_t* q16;
  uint16_t* weights;
};

// Caller buffers of the cross-channel 3x3 maps (device pointers).
struct CrossBufs {
  uint64_t* cross;    // [K][2][NB][3] = (S_RG, S_RB, S_GB)
  double* params3;    // [K][2][NB][12] = M row-major, then t
  uint8_t* valid3;    // [K][2][NB]
  int64_t* q3;        // [K][2][NB][12]
  uint16_t* weights;  // [K][w_max]
};

// Context-wide constants passed to every kernel.
struct Geo {
  const DevCam* cams;    // device array [K]
  const Tile* tiles;     // device array [n_tiles], camera-major
  const int32_t* wg_seg; // device array [n_wg + 1]: workgroup w takes segments [wg_seg[w], wg_seg[w + 1])
  int32_t n_cams, n_blocks, w_max, n_tiles;
  int32_t mode;
  int32_t n_wg;          // apply workgroups
  double alpha, a_min, a_max;
  uint64_t active;       // cameras processed by this launch (bit k = camera k)
  int32_t vblend;        // 1: the maps of adjacent blocks are blended row by row in the apply
  int32_t fit;           // RT_FIT_MOMENTS or RT_FIT_QUANTILE
};

__host__ __device__ inline bool cam_active(const Geo& g, int k) { return (g.active >> k) & 1ull; }

// Buffer resource over one frame: loads beyond the last sample of the frame
// return zero and stores there are dropped by the hardware range check.
constexpr int kRsrcWord3 = 0x00020000;   // raw dword access on gfx9-family parts

// Values the caller knows to be the same in every lane of the wave, moved to
// scalar registers.  Table entries read from global memory land in vector
// registers; without this a buffer resource built from them would be
// non-uniform and every access through it would be wrapped in a loop over
// the distinct values.
__device__ inline int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uniform(int64_t v) {
  const uint64_t u = (uint64_t)v;
  return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(u >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)u));
}
template <typename T>
__device__ inline T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform((int64_t)reinterpret_cast<uintptr_t>(p)));
}

__device__ inline DevCam uniform_cam(const DevCam& c) {
  DevCam u;
  u.width = uniform(c.width); u.height = uniform(c.height); u.channels = uniform(c.channels);
  u.bit_depth = uniform(c.bit_depth); u.bps = uniform(c.bps); u.band = uniform(c.band); u.half = uniform(c.half);
  u.row_bytes = uniform(c.row_bytes);
  u.face_cam[0] = uniform(c.face_cam[0]); u.face_cam[1] = uniform(c.face_cam[1]);
  u.face_side[0] = uniform(c.face_side[0]); u.face_side[1] = uniform(c.face_side[1]);
  u.tile_begin = uniform(c.tile_begin); u.tile_end = uniform(c.tile_end);
  u.pitch = uniform(c.pitch);
  return u;
}

__device__ inline Tile uniform_tile(const Tile& t) {
  return Tile{uniform(t.cam), uniform(t.block), uniform(t.r0), uniform(t.r1)};
}

// p and cam must be uniform over the wave (see uniform_cam).
__device__ inline __amdgpu_buffer_rsrc_t frame_rsrc(const void* p, const DevCam& cam) {
  const int64_t bytes = (int64_t)(cam.height - 1) * cam.pitch + cam.row_bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(uniform_ptr(p)), (short)0, uniform((int32_t)bytes),
                                           kRsrcWord3);
}

// Index of a (camera, side, block, channel) unit in the caller layouts.
__host__ __device__ inline int64_t unit_index(int k, int s, int j, int c, int nb) {
  return (((int64_t)k * 2 + s) * nb + j) * kCS + c;
}

// Launchers (each defined next to its kernels).  All return hipError_t of the launch.
hipError_t launch_band_stats(const Geo& g, const FramePtrs& fp, const Bufs& b, hipStream_t st);
hipError_t launch_estimate(const Geo& g, const Bufs& b, hipStream_t st);
hipError_t launch_band_estimate(const Geo& g, const FramePtrs& fp, const Bufs& b, hipStream_t st);
hipError_t launch_build_lut(const Geo& g, const Bufs& b, hipStream_t st);
hipError_t launch_apply(const Geo& g, const FramePtrs& fp, const Bufs& b, bool write, bool stats, hipStream_t st,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Host addresses of the kernels that launch_band_estimate and launch_apply
// launch for g (the latter with write and stats as given); both take
// (Geo, FramePtrs, Bufs).  Used to find them among a captured graph's nodes.
const void* band_estimate_kernel(const Geo& g);
const void* apply_kernel(const Geo& g, bool write, bool stats);

// Apply with whole-frame statistics of sp.n_sets (1..kSetsMax) frame-sets of
// the rig in one launch (every camera at most kSetCams; g.active the same
// for all sets).
hipError_t launch_apply_sets(const Geo& g, const SetPtrs& sp, hipStream_t st, hipEvent_t start = nullptr,
                             hipEvent_t stop = nullptr);
hipError_t launch_zero_whole(const Geo& g, const Bufs& b, hipStream_t st);
hipError_t launch_weights(const Geo& g, const Bufs& b, hipStream_t st);
hipError_t launch_cross_stats(const Geo& g, const FramePtrs& fp, const CrossBufs& x, hipStream_t st);
hipError_t launch_estimate_cross(const Geo& g, const Bufs& b, const CrossBufs& x, hipStream_t st);
hipError_t launch_build_cross(const Geo& g, const CrossBufs& x, hipStream_t st);
hipError_t launch_apply_cross(const Geo& g, const FramePtrs& fp, const Bufs& b, const CrossBufs& x, bool stats,
                              hipStream_t st);
struct PrevPtrs;
struct Removal;
hipError_t launch_band_estimate_removal(const Geo& g, const FramePtrs& fp, const PrevPtrs& pp, const Bufs& b,
                                        const Removal& rm, hipStream_t st);
hipError_t launch_motion_stats(const Geo& g, const FramePtrs& fp, const PrevPtrs& pp, const Bufs& b,
                               const Removal& rm, hipStream_t st);
hipError_t launch_estimate_removal(const Geo& g, const Bufs& b, const Removal& rm, hipStream_t st);
hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, int vec_bytes, hipStream_t st);
hipError_t launch_attention(const Geo& g, const FramePtrs& fp, const uint8_t* const* prev, uint32_t* cells,
                            uint32_t* windows, uint8_t* selected, int hc, int wc, int cell, int m, uint32_t tau,
                            uint32_t theta, hipStream_t st);
hipError_t launch_seam_cost(const Geo& g, const FramePtrs& fp, double* seam, double* interior, double* rows,
                            int row_stride, int factor, int max_rows, hipStream_t st);

}  // namespace rc
