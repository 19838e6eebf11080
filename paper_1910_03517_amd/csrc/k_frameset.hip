// DISABLED - not compiled into the library.  This single-launch variant of
// the frame-set (a work queue with in-kernel dependency waits) did not
// complete on its first two runs on the device and stays switched off until
// the cause is found; rt_frameset enqueues the four kernels of k_stats.hip,
// k_estimate.hip and k_apply.hip instead.  Kept as the design record.
//
// One persistent launch per frame-set: band statistics -> estimate and tables
// -> apply with fused statistics -> whole-frame reduction (section 3.1, with
// the statistics of frame t correcting frame t).
//
// Work items, claimed in increasing order from one atomic counter:
//   [0, U)        band statistics of unit (camera, side, block), U = K * 2 * NB
//   [U, 2U)       estimate + tables of unit (camera, side, block)
//   [2U, 2U + T)  apply of tile t (camera-major)
// An item only ever waits for items with smaller numbers: estimate waits for
// the band statistics of its own and its facing band, a tile waits for the
// tables of both sides of its block.  Those items were claimed earlier by
// workgroups that are running, so the queue cannot deadlock whatever the
// number of resident workgroups.  Completion flags hold the launch's epoch + 1
// and never need clearing.  The last tile of a camera sums the camera's tile
// histograms.  Every wait is bounded by a wall-clock budget: on expiry it
// raises the context's error word and carries on (later waits then return at
// once), so a bug shows as an error, never as a hang.
//
// Cache maintenance is kept to one release per produced item and one acquire
// per consumed item: polls are relaxed loads, because an acquire load in a
// polling loop would invalidate the L2 on every iteration.
//
// Sync words (uint32, context scratch, zero at creation):
//   [0] work counter  [1] exit counter  [2] epoch  [3] error
//   [4, 4+K) tiles done per camera  [4+K, 4+K+U) band flags  [4+K+U, 4+K+2U) table flags
#include "dev_apply.h"
#include "dev_stats.h"

namespace rc {

constexpr int kSpinLimit = 1 << 20;   // poll cap; the wall-clock budget normally ends a failed wait first

union FramesetLds {
  StatsLds s;
  ApplyLds a;
};

__device__ inline uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_relaxed(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by one thread: wait until *f == target, then acquire.  Polls are
// relaxed loads (no cache maintenance); the single acquire fence after the
// flag is seen makes the producer's data visible.  The wait is bounded by a
// wall-clock budget; once any wait of the launch has expired, all later waits
// return at once.
__device__ inline void wait_flag(const uint32_t* f, uint32_t target, uint32_t* err, uint64_t budget_ticks) {
  const uint64_t t0 = wall_clock64();
  for (int it = 0; it < kSpinLimit; ++it) {
    if (ld_relaxed(f) == target) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return;
    }
    if (ld_relaxed(err) != 0u) return;
    if (wall_clock64() - t0 > budget_ticks) break;
    __builtin_amdgcn_s_sleep(4);
  }
  st_relaxed(err, 1u);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Wait for this wave's outstanding global loads and stores (vmcnt(0) on the
// gfx9 family, where stores are counted by vmcnt).
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Every wave waits for its own global stores of this item, the barrier then
// orders them before thread 0's single release, which publishes them with the flag.
__device__ inline void publish(uint32_t* f, uint32_t target) {
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kThreads) void k_frameset(Geo g, FramePtrs fp, Bufs b, uint64_t budget_ticks) {
  __shared__ FramesetLds L;
  __shared__ int s_item;
  __shared__ uint32_t s_epoch;
  __shared__ int s_last;
  const int tid = threadIdx.x;
  uint32_t* sync = g.scr.sync;
  const int K = g.n_cams, nb = g.n_blocks;
  const int U = K * 2 * nb;
  uint32_t* done = sync + 4;
  uint32_t* flag_band = sync + 4 + K;
  uint32_t* flag_lut = flag_band + U;
  uint32_t* err = sync + 3;
  const int n_items = 2 * U + g.n_tiles;

  if (tid == 0) s_epoch = __hip_atomic_load(sync + 2, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t target = __builtin_amdgcn_readfirstlane(s_epoch) + 1;

  for (;;) {
    if (tid == 0) s_item = (int)__hip_atomic_fetch_add(sync + 0, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: keep item state in SGPRs
    __syncthreads();
    if (item >= n_items) break;

    if (item < U) {
      band_unit_dispatch(g, fp, b, item, L.s);
      publish(flag_band + item, target);
    } else if (item < 2 * U) {
      const int u3 = item - U;                 // (k * 2 + s) * nb + j
      const int k = u3 / (2 * nb);
      const int s = (u3 / nb) & 1;
      const int j = u3 % nb;
      const DevCam& cam = g.cams[k];
      if (tid == 0) {
        wait_flag(flag_band + u3, target, err, budget_ticks);
        const int fc = cam.face_cam[s];
        if (fc >= 0) wait_flag(flag_band + (fc * 2 + cam.face_side[s]) * nb + j, target, err, budget_ticks);
      }
      __syncthreads();
      if (tid < kCS) estimate_unit(g, b, u3 * kCS + tid);
      __syncthreads();
      lut_entry(g, b, u3, tid);
      if (s == 0 && j == 0)                    // the context's weight table, written once per camera
        for (int col = tid; col < g.w_max; col += kThreads)
          b.weights[(int64_t)k * g.w_max + col] = (uint16_t)blend_weight(cam.width, col);
      publish(flag_lut + u3, target);
    } else {
      const int ti = item - 2 * U;
      const Tile t = g.tiles[ti];
      if (tid == 0) {
        wait_flag(flag_lut + (t.cam * 2 + 0) * nb + t.block, target, err, budget_ticks);
        wait_flag(flag_lut + (t.cam * 2 + 1) * nb + t.block, target, err, budget_ticks);
      }
      __syncthreads();
      apply_tile_dispatch<true, true, false>(g, fp, b, ti, L.a);
      wait_vmem();
      __syncthreads();
      if (tid == 0) {
        const DevCam& cam = g.cams[t.cam];
        const uint32_t n = (uint32_t)(cam.tile_end - cam.tile_begin);
        const uint32_t old = __hip_atomic_fetch_add(done + t.cam, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (old + 1 == n);
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(s_last)) {
        whole_reduce_cam(g, b, t.cam, L.s);
        if (tid == 0) st_relaxed(done + t.cam, 0u);
      }
      __syncthreads();
    }
  }

  // The last workgroup out resets the counters and advances the epoch.
  if (tid == 0) {
    const uint32_t old = __hip_atomic_fetch_add(sync + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == gridDim.x) {
      st_relaxed(sync + 0, 0u);
      st_relaxed(sync + 1, 0u);
      __hip_atomic_store(sync + 2, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

int frameset_max_grid() {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_frameset, kThreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  cached = cus * per_cu;
  return cached;
}

// Wall-clock ticks a single dependency wait may take before it is declared
// failed: 50 ms, far above any legitimate wait of one frame-set.
static uint64_t wait_budget_ticks() {
  static uint64_t cached = 0;
  if (cached) return cached;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      khz <= 0)
    khz = 100000;
  cached = (uint64_t)khz * 50;
  return cached;
}

hipError_t launch_frameset(const Geo& g, const FramePtrs& fp, const Bufs& b, int grid, hipStream_t st) {
  const int n_items = 2 * g.n_cams * 2 * g.n_blocks + g.n_tiles;
  if (grid <= 0) grid = frameset_max_grid();
  if (grid > n_items) grid = n_items;
  hipLaunchKernelGGL(k_frameset, dim3(grid), dim3(kThreads), 0, st, g, fp, b, wait_budget_ticks());
  return hipGetLastError();
}

}  // namespace rc
