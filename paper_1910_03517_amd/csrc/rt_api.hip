// Host side of the C-ABI: rig validation, context tables, argument checks and
// the launch sequences of every entry point.  No exception leaves this file.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "dev_motion.h"
#include "rt_ahead_internal.h"
#include "rt_internal.h"
#include "rt_surrogate_internal.h"

using namespace rc;

struct rt_ctx {
  int device = 0;
  int n_cams = 0;
  rt_opts opts{};
  std::vector<rt_camera_desc> cams;
  std::vector<DevCam> hcams;
  std::vector<Tile> htiles;
  int w_max = 0;
  int tile_rows = 0;
  int grid = 0;             // apply workgroups (0 = one per tile)
  DevCam* dcams = nullptr;
  Tile* dtiles = nullptr;
  int32_t* dwg = nullptr;   // [n_wg + 1] first segment of each apply workgroup
  double* seam_rows = nullptr;   // row values of rt_seam_cost when the caller passes none
  size_t seam_rows_n = 0;

  // Optional timing of the apply kernel: events recorded right before and
  // after each apply launch, in a ring of n_timing slots.
  int n_timing = 0;
  int timing_every = 1;
  int64_t n_timed = 0;
  int64_t n_applies = 0;
  std::vector<hipEvent_t> ev_begin, ev_end;
  std::vector<int32_t> timed_sets;   // frame-sets each timed launch covered
  bool capturing = false;   // no timing events inside a captured graph
  int64_t generation = 0;   // bumped whenever device tables are rebuilt
  Geo geo{};
};

struct rt_graph {
  rt_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t generation = 0;
  bool pipelined = false;
  // Kernel nodes whose second argument is a FramePtrs: next = false for
  // the frame-set's own frames (frames -> out_frames), true for next_frames.
  struct FrameNode {
    hipGraphNode_t node;
    bool next;
  };
  std::vector<FrameNode> frame_nodes;
};



namespace {

thread_local std::string g_last_error;

rt_status fail(rt_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
rt_status fail(rt_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

rt_status hip_fail(hipError_t e, const char* what) {
  return fail(RT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr int kMaxDim = 32768;
constexpr int kDefaultTileRows = 32;
constexpr int kMaxApplyGrid = 1 << 16;

bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

// Frames of the cameras in `active` only (the others may be NULL).
rt_status check_frames_masked(const rt_ctx* ctx, uint64_t active, const void* const* frames, const char* name) {
  if (!frames) return fail(RT_EINVAL, "%s is NULL", name);
  for (int k = 0; k < ctx->n_cams; ++k) {
    if (!((active >> k) & 1ull)) continue;
    if (!frames[k]) return fail(RT_EINVAL, "%s[%d] is NULL", name, k);
    if (!aligned(frames[k], 16)) return fail(RT_EINVAL, "%s[%d] is not 16-byte aligned", name, k);
  }
  return RT_OK;
}

// Frames of the context's active cameras.
rt_status check_frames(const rt_ctx* ctx, const void* const* frames, const char* name) {
  return check_frames_masked(ctx, ctx->geo.active, frames, name);
}

rt_status check_ptr(const void* p, uintptr_t align, const char* name) {
  if (!p) return fail(RT_EINVAL, "%s is NULL", name);
  if (!aligned(p, align)) return fail(RT_EINVAL, "%s is not %u-byte aligned", name, (unsigned)align);
  return RT_OK;
}

FramePtrs make_ptrs_masked(const rt_ctx* ctx, const void* const* in, void* const* out, uint64_t active) {
  FramePtrs fp;
  memset(&fp, 0, sizeof fp);
  for (int k = 0; k < ctx->n_cams; ++k) {
    if (!((active >> k) & 1ull)) continue;
    fp.in[k] = (const uint8_t*)in[k];
    fp.out[k] = out ? (uint8_t*)out[k] : nullptr;
  }
  return fp;
}

FramePtrs make_ptrs(const rt_ctx* ctx, const void* const* in, void* const* out) {
  return make_ptrs_masked(ctx, in, out, ctx->geo.active);
}

uint64_t all_cams(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// A non-empty set of whole rings within the context.
rt_status check_active(const rt_ctx* ctx, uint64_t active) {
  if (active == 0) return fail(RT_EINVAL, "active is empty");
  if (active & ~all_cams(ctx->n_cams)) return fail(RT_EINVAL, "active names cameras beyond n_cams = %d", ctx->n_cams);
  // A seam's estimate reads both of its bands, so a ring is active as a whole.
  for (int k = 0; k < ctx->n_cams; ++k) {
    if (!((active >> k) & 1ull)) continue;
    for (int i = 0; i < ctx->n_cams; ++i)
      if (ctx->cams[i].ring == ctx->cams[k].ring && !((active >> i) & 1ull))
        return fail(RT_EINVAL, "active holds camera %d of ring %d but not camera %d of the same ring", k,
                    ctx->cams[k].ring, i);
  }
  return RT_OK;
}

}  // namespace

// Tile table and device tables.  Every block is split into
// ceil(rows / cap) tiles of equal height (+-1 row), cap = tile_rows or less
// where the apply pass's packed histogram needs it; tiles are camera-major.
// Apply work.  grid == 0: every vertical block of every camera is cut into
// ceil(rows / cap) tiles of equal height (+-1 row), one workgroup per tile.
// grid > 0: `grid` workgroups, each on a contiguous share of rows, the
// shares as even in bytes as whole cameras allow, cut into segments at block
// boundaries and at most cap rows.  cap = tile_rows, or less where the packed
// histogram needs it.
static rt_status build_tables(rt_ctx* ctx, int tile_rows, int grid) {
  const int n_cams = ctx->n_cams;
  const int nb = ctx->opts.n_blocks;
  ctx->tile_rows = tile_rows;
  ctx->grid = grid;
  ++ctx->generation;
  ctx->htiles.clear();
  // Rows [a, e) of camera k, cut at block boundaries and at most cap rows.
  auto emit = [&](int k, int a, int e) {
    const int H = ctx->cams[k].height;
    const int cap = std::min(tile_rows, max_tile_rows(ctx->cams[k].width));
    for (int j = 0; j < nb; ++j) {
      const int b0 = std::max(a, (int)((int64_t)j * H / nb)), b1 = std::min(e, (int)((int64_t)(j + 1) * H / nb));
      const int rows = b1 - b0;
      if (rows <= 0) continue;
      const int parts = (rows + cap - 1) / cap;
      for (int p = 0; p < parts; ++p)
        ctx->htiles.push_back(
            Tile{k, j, b0 + (int)((int64_t)p * rows / parts), b0 + (int)((int64_t)(p + 1) * rows / parts)});
    }
  };
  std::vector<int32_t> wg;
  int G = 0;
  if (grid == 0) {
    for (int k = 0; k < n_cams; ++k) emit(k, 0, ctx->cams[k].height);
    G = (int)ctx->htiles.size();
    wg.resize(G + 1);
    for (int w = 0; w <= G; ++w) wg[w] = w;
  } else if (grid >= n_cams) {
    // Every camera gets a whole number of shares, one plus its part of the
    // other G - K by bytes (largest remainders), and its rows are split
    // evenly among them: no share spans two cameras.
    G = grid;
    int64_t total = 0;
    for (int k = 0; k < n_cams; ++k) total += (int64_t)ctx->cams[k].height * ctx->hcams[k].row_bytes;
    std::vector<int> n(n_cams, 1);
    std::vector<std::pair<int64_t, int>> rem(n_cams);
    int given = n_cams;
    for (int k = 0; k < n_cams; ++k) {
      const __int128 q = (__int128)(G - n_cams) * ((int64_t)ctx->cams[k].height * ctx->hcams[k].row_bytes);
      n[k] += (int)(q / total);
      given += (int)(q / total);
      rem[k] = {(int64_t)(q % total), -k};
    }
    std::sort(rem.begin(), rem.end(), std::greater<std::pair<int64_t, int>>());
    for (int i = 0; given < G; ++i, ++given) ++n[-rem[i].second];
    wg.resize(G + 1);
    int w = 0;
    for (int k = 0; k < n_cams; ++k) {
      const int H = ctx->cams[k].height;
      for (int i = 0; i < n[k]; ++i, ++w) {
        wg[w] = (int32_t)ctx->htiles.size();
        emit(k, (int)((int64_t)i * H / n[k]), (int)((int64_t)(i + 1) * H / n[k]));
      }
    }
  } else {
    // Fewer workgroups than cameras: share w starts at the first row whose
    // byte offset reaches w / G of the total, so shares span cameras.
    G = grid;
    std::vector<int64_t> base(n_cams + 1, 0);
    for (int k = 0; k < n_cams; ++k)
      base[k + 1] = base[k] + (int64_t)ctx->cams[k].height * ctx->hcams[k].row_bytes;
    auto share_start = [&](int w, int& cam, int& row) {
      const int64_t target = (int64_t)((__int128)w * base[n_cams] / G);
      cam = 0;
      while (cam < n_cams && base[cam + 1] <= target) ++cam;
      if (cam == n_cams) { row = 0; return; }
      const int64_t rb = ctx->hcams[cam].row_bytes;
      row = (int)((target - base[cam] + rb - 1) / rb);
      if (row >= ctx->cams[cam].height) { ++cam; row = 0; }
    };
    wg.resize(G + 1);
    int c0, r0s;
    share_start(0, c0, r0s);
    for (int w = 0; w < G; ++w) {
      int c1, r1s;
      share_start(w + 1, c1, r1s);
      wg[w] = (int32_t)ctx->htiles.size();
      for (int k = c0; k <= c1 && k < n_cams; ++k) emit(k, k == c0 ? r0s : 0, k == c1 ? r1s : ctx->cams[k].height);
      c0 = c1;
      r0s = r1s;
    }
  }
  wg[G] = (int32_t)ctx->htiles.size();
  for (int k = 0; k < n_cams; ++k) ctx->hcams[k].tile_begin = ctx->hcams[k].tile_end = 0;
  for (size_t i = ctx->htiles.size(); i-- > 0;) {
    DevCam& d = ctx->hcams[ctx->htiles[i].cam];
    if (d.tile_end == 0) d.tile_end = (int32_t)i + 1;
    d.tile_begin = (int32_t)i;
  }
  const size_t nt = ctx->htiles.size();
  if (ctx->dtiles) (void)hipFree(ctx->dtiles);
  if (ctx->dwg) (void)hipFree(ctx->dwg);
  ctx->dtiles = nullptr;
  ctx->dwg = nullptr;
  hipError_t e = hipSuccess;
  if (!ctx->dcams) e = hipMalloc((void**)&ctx->dcams, sizeof(DevCam) * n_cams);
  if (e == hipSuccess) e = hipMalloc((void**)&ctx->dtiles, sizeof(Tile) * std::max<size_t>(nt, 1));
  if (e == hipSuccess) e = hipMalloc((void**)&ctx->dwg, sizeof(int32_t) * wg.size());
  if (e != hipSuccess) return fail(RT_ENOMEM, "device tables: %s", hipGetErrorString(e));
  e = hipMemcpy(ctx->dcams, ctx->hcams.data(), sizeof(DevCam) * n_cams, hipMemcpyHostToDevice);
  if (e == hipSuccess && nt) e = hipMemcpy(ctx->dtiles, ctx->htiles.data(), sizeof(Tile) * nt, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->dwg, wg.data(), sizeof(int32_t) * wg.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "uploading context tables");
  Geo& g = ctx->geo;
  g.cams = ctx->dcams;
  g.tiles = ctx->dtiles;
  g.wg_seg = ctx->dwg;
  g.n_wg = G;
  g.n_cams = n_cams;
  g.n_blocks = nb;
  g.w_max = ctx->w_max;
  g.n_tiles = (int32_t)nt;
  g.mode = ctx->opts.mode;
  g.vblend = ctx->opts.vblend;
  g.fit = ctx->opts.fit;
  g.alpha = ctx->opts.ema_alpha;
  g.a_min = ctx->opts.a_min;
  g.a_max = ctx->opts.a_max;
  if (g.active == 0) g.active = all_cams(n_cams);
  return RT_OK;
}

extern "C" {

const char* rt_status_str(rt_status s) {
  switch (s) {
    case RT_OK: return "ok";
    case RT_EINVAL: return "invalid argument";
    case RT_ENOMEM: return "out of device memory";
    case RT_EDEVICE: return "HIP device error";
    case RT_EUNSUPPORTED: return "unsupported";
    case RT_ESTATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* rt_last_error(void) { return g_last_error.c_str(); }

static hipError_t static_scratch(int device, void** out);

rt_status rt_ctx_create(const rt_camera_desc* cams, int32_t n_cams, const rt_opts* opts, rt_ctx** out) {
  if (!out) return fail(RT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cams || !opts) return fail(RT_EINVAL, "cams or opts is NULL");
  if (n_cams < 1 || n_cams > RT_MAX_CAMS) return fail(RT_EINVAL, "n_cams %d outside 1..%d", n_cams, RT_MAX_CAMS);
  const rt_opts& o = *opts;
  if (o.n_blocks < 1 || o.n_blocks > RT_MAX_BLOCKS) return fail(RT_EINVAL, "n_blocks %d outside 1..%d", o.n_blocks, RT_MAX_BLOCKS);
  if (o.band_width < 1) return fail(RT_EINVAL, "band_width %d < 1", o.band_width);
  if (o.closed_ring != 0 && o.closed_ring != 1) return fail(RT_EINVAL, "closed_ring must be 0 or 1");
  if (o.mode != RT_MODE_STANDARD && o.mode != RT_MODE_SMOOTHING) return fail(RT_EINVAL, "mode %d unknown", o.mode);
  if (!(o.ema_alpha > 0.0 && o.ema_alpha <= 1.0)) return fail(RT_EINVAL, "ema_alpha must lie in (0, 1]");
  if (!(o.a_min > 0.0 && o.a_min <= o.a_max && isfinite(o.a_max)))
    return fail(RT_EINVAL, "need 0 < a_min <= a_max < inf");
  if (o.vblend != 0 && o.vblend != 1) return fail(RT_EINVAL, "vblend must be 0 or 1");
  if (o.fit != RT_FIT_MOMENTS && o.fit != RT_FIT_QUANTILE) return fail(RT_EINVAL, "fit %d unknown", o.fit);
  if (o.vblend)
    for (int k = 0; k < n_cams; ++k)
      if (cams[k].height < o.n_blocks)
        return fail(RT_EUNSUPPORTED, "vblend needs blocks of at least one row: camera %d has %d rows < n_blocks %d", k,
                    cams[k].height, o.n_blocks);

  for (int k = 0; k < n_cams; ++k) {
    const rt_camera_desc& c = cams[k];
    if (c.width < 1 || c.height < 1 || c.width > kMaxDim || c.height > kMaxDim)
      return fail(RT_EINVAL, "camera %d: size %dx%d outside 1..%d", k, c.width, c.height, kMaxDim);
    if (c.channels != 1 && c.channels != 3) return fail(RT_EINVAL, "camera %d: channels %d not 1 or 3", k, c.channels);
    if (c.bit_depth < 8 || c.bit_depth > 16) return fail(RT_EINVAL, "camera %d: bit_depth %d outside 8..16", k, c.bit_depth);
    if (c.bit_depth > 8 && c.channels != 1)
      return fail(RT_EINVAL, "camera %d: 16-bit samples need channels == 1", k);
    const int64_t row_bytes = (int64_t)c.width * c.channels * (c.bit_depth > 8 ? 2 : 1);
    if (c.pitch_bytes < row_bytes || c.pitch_bytes % 16 != 0)
      return fail(RT_EINVAL, "camera %d: pitch %lld must be >= %lld and a multiple of 16", k,
                  (long long)c.pitch_bytes, (long long)row_bytes);
    if ((int64_t)(c.height - 1) * c.pitch_bytes + row_bytes >= (int64_t)1 << 31)
      return fail(RT_EUNSUPPORTED, "camera %d: frame larger than 2 GiB", k);
  }
  // Rings: positions 0..m-1 each once; equal channels and bit depth.
  for (int k = 0; k < n_cams; ++k) {
    int m = 0;
    std::vector<int> seen;
    for (int i = 0; i < n_cams; ++i) {
      if (cams[i].ring != cams[k].ring) continue;
      ++m;
      seen.push_back(cams[i].pos);
      if (cams[i].channels != cams[k].channels || cams[i].bit_depth != cams[k].bit_depth)
        return fail(RT_EINVAL, "ring %d mixes channel counts or bit depths", cams[k].ring);
    }
    std::sort(seen.begin(), seen.end());
    for (int p = 0; p < m; ++p)
      if (seen[p] != p) return fail(RT_EINVAL, "ring %d: positions must be 0..%d, each once", cams[k].ring, m - 1);
  }

  rt_ctx* ctx = new (std::nothrow) rt_ctx();
  if (!ctx) return fail(RT_ENOMEM, "host allocation failed");
  (void)hipGetDevice(&ctx->device);
  {
    // Set-up of the static workspace on this device (rt_surrogate_frameset_static);
    // a failure is kept and reported by that entry point only.
    void* unused = nullptr;
    (void)static_scratch(ctx->device, &unused);
  }
  ctx->n_cams = n_cams;
  ctx->opts = o;
  ctx->cams.assign(cams, cams + n_cams);
  ctx->tile_rows = kDefaultTileRows;
  ctx->hcams.resize(n_cams);
  for (int k = 0; k < n_cams; ++k) {
    const rt_camera_desc& c = cams[k];
    DevCam& d = ctx->hcams[k];
    memset(&d, 0, sizeof d);
    d.width = c.width;
    d.height = c.height;
    d.channels = c.channels;
    d.bit_depth = c.bit_depth;
    d.bps = c.bit_depth > 8 ? 2 : 1;
    d.half = c.width / 2;
    d.band = std::min(o.band_width, d.half);
    d.row_bytes = c.width * c.channels * d.bps;
    d.pitch = c.pitch_bytes;
    // Ring neighbours: right side of position p meets the left side of p + 1.
    int m = 0;
    for (int i = 0; i < n_cams; ++i) m += cams[i].ring == c.ring;
    for (int s = 0; s < 2; ++s) {
      int q = c.pos + (s == 1 ? 1 : -1);
      d.face_cam[s] = -1;
      d.face_side[s] = 1 - s;
      if (q < 0 || q >= m) {
        if (!o.closed_ring) continue;
        q = (q + m) % m;
      }
      for (int i = 0; i < n_cams; ++i)
        if (cams[i].ring == c.ring && cams[i].pos == q) d.face_cam[s] = i;
    }
    ctx->w_max = std::max(ctx->w_max, c.width);
  }
  rt_status st = build_tables(ctx, kDefaultTileRows, 0);
  if (st != RT_OK) {
    rt_ctx_destroy(ctx);
    return st;
  }
  *out = ctx;
  return RT_OK;
}

static void free_timing(rt_ctx* ctx) {
  for (hipEvent_t ev : ctx->ev_begin) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : ctx->ev_end) (void)hipEventDestroy(ev);
  ctx->ev_begin.clear();
  ctx->ev_end.clear();
  ctx->timed_sets.clear();
  ctx->n_timing = 0;
  ctx->n_timed = 0;
}

rt_status rt_ctx_destroy(rt_ctx* ctx) {
  if (!ctx) return RT_OK;
  (void)hipDeviceSynchronize();
  free_timing(ctx);
  if (ctx->dcams) (void)hipFree(ctx->dcams);
  if (ctx->dtiles) (void)hipFree(ctx->dtiles);
  if (ctx->dwg) (void)hipFree(ctx->dwg);
  if (ctx->seam_rows) (void)hipFree(ctx->seam_rows);
  delete ctx;
  return RT_OK;
}

rt_status rt_ctx_sizes(const rt_ctx* ctx, rt_sizes* out) {
  if (!ctx || !out) return fail(RT_EINVAL, "ctx or out is NULL");
  const int64_t K = ctx->n_cams, NB = ctx->opts.n_blocks;
  out->n_cams = ctx->n_cams;
  out->n_blocks = ctx->opts.n_blocks;
  out->w_max = ctx->w_max;
  out->reserved = 0;
  out->band_hist = K * 2 * NB * kCS * kNB;
  out->band_sums = K * 2 * NB * kCS * 3;
  out->whole_hist = K * kCS * kNB;
  out->whole_sums = K * kCS * 3;
  out->params = K * 2 * NB * kCS * 2;
  out->valid = K * 2 * NB * kCS;
  out->lut8 = K * 2 * NB * kCS * kNB;
  out->q16 = K * 2 * NB * kCS * 2;
  out->weights = K * ctx->w_max;
  return RT_OK;
}

static rt_status check_stats(const rt_stats_buf* s, bool bands, bool whole) {
  if (!s) return fail(RT_EINVAL, "stats buffer struct is NULL");
  rt_status r = RT_OK;
  if (bands && (r = check_ptr(s->band_hist, 4, "band_hist")) != RT_OK) return r;
  if (bands && (r = check_ptr(s->band_sums, 8, "band_sums")) != RT_OK) return r;
  if (whole && (r = check_ptr(s->whole_hist, 4, "whole_hist")) != RT_OK) return r;
  if (whole && (r = check_ptr(s->whole_sums, 8, "whole_sums")) != RT_OK) return r;
  return RT_OK;
}

static rt_status check_params(const rt_params_buf* p) {
  if (!p) return fail(RT_EINVAL, "params buffer struct is NULL");
  rt_status r = check_ptr(p->params, 8, "params");
  if (r == RT_OK) r = check_ptr(p->valid, 1, "valid");
  return r;
}

static rt_status check_lut(const rt_lut_buf* l) {
  if (!l) return fail(RT_EINVAL, "lut buffer struct is NULL");
  rt_status r = check_ptr(l->lut8, 4, "lut8");
  if (r == RT_OK) r = check_ptr(l->q16, 8, "q16");
  if (r == RT_OK) r = check_ptr(l->weights, 2, "weights");
  return r;
}

static Bufs make_bufs(const rt_stats_buf* s, const rt_params_buf* p, const rt_lut_buf* l) {
  Bufs b;
  memset(&b, 0, sizeof b);
  if (s) { b.band_hist = s->band_hist; b.band_sums = s->band_sums; b.whole_hist = s->whole_hist; b.whole_sums = s->whole_sums; }
  if (p) { b.params = p->params; b.valid = p->valid; }
  if (l) { b.lut8 = l->lut8; b.q16 = l->q16; b.weights = l->weights; }
  return b;
}

// The apply kernel, its dispatch timed by the context's events when enabled
// (never inside a graph capture).
static hipError_t timed_apply(rt_ctx* ctx, const Geo& g, const FramePtrs& fp, const Bufs& b, bool write,
                              bool stats, hipStream_t st) {
  if (ctx->n_timing <= 0 || ctx->capturing) return launch_apply(g, fp, b, write, stats, st);
  if (ctx->n_applies++ % ctx->timing_every != 0) return launch_apply(g, fp, b, write, stats, st);
  const int slot = (int)(ctx->n_timed % ctx->n_timing);
  const hipError_t e = launch_apply(g, fp, b, write, stats, st, ctx->ev_begin[slot], ctx->ev_end[slot]);
  if (e == hipSuccess) ctx->timed_sets[slot] = 1, ++ctx->n_timed;
  return e;
}

// The same for an apply launch over several frame-sets.
static hipError_t timed_apply_sets(rt_ctx* ctx, const Geo& g, const SetPtrs& sp, hipStream_t st) {
  if (ctx->n_timing <= 0 || ctx->capturing) return launch_apply_sets(g, sp, st);
  if (ctx->n_applies++ % ctx->timing_every != 0) return launch_apply_sets(g, sp, st);
  const int slot = (int)(ctx->n_timed % ctx->n_timing);
  const hipError_t e = launch_apply_sets(g, sp, st, ctx->ev_begin[slot], ctx->ev_end[slot]);
  if (e == hipSuccess) ctx->timed_sets[slot] = sp.n_sets, ++ctx->n_timed;
  return e;
}

// Apply (or statistics only) with fused whole-frame statistics, accumulated
// by the tiles into the whole-frame buffers.  zero_first clears them first
// (the frame-set path clears them in its estimate kernel instead).
static rt_status whole_pass(rt_ctx* ctx, const Geo& g, const FramePtrs& fp, const Bufs& b, bool write,
                            bool zero_first, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (zero_first) e = launch_zero_whole(g, b, st);
  if (e != hipSuccess) return hip_fail(e, "clearing whole-frame statistics");
  e = timed_apply(ctx, g, fp, b, write, true, st);
  if (e != hipSuccess) return hip_fail(e, write ? "apply" : "whole-frame statistics");
  return RT_OK;
}

rt_status rt_stats(rt_ctx* ctx, const void* const* frames, const rt_stats_buf* out, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_frames(ctx, frames, "frames");
  if (r != RT_OK) return r;
  if (!out) return fail(RT_EINVAL, "out is NULL");
  const bool whole = out->whole_hist && out->whole_sums;
  if ((r = check_stats(out, true, whole)) != RT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const FramePtrs fp = make_ptrs(ctx, frames, nullptr);
  const Bufs b = make_bufs(out, nullptr, nullptr);
  hipError_t e = launch_band_stats(ctx->geo, fp, b, st);
  if (e != hipSuccess) return hip_fail(e, "band statistics");
  if (whole) return whole_pass(ctx, ctx->geo, fp, b, false, true, st);
  return RT_OK;
}

rt_status rt_estimate(rt_ctx* ctx, const rt_stats_buf* stats, const rt_params_buf* state, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_stats(stats, true, false);
  if (r == RT_OK) r = check_params(state);
  if (r != RT_OK) return r;
  hipError_t e = launch_estimate(ctx->geo, make_bufs(stats, state, nullptr), (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "estimate");
}

rt_status rt_build_lut(rt_ctx* ctx, const rt_params_buf* params, const rt_lut_buf* out, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_params(params);
  if (r == RT_OK) r = check_lut(out);
  if (r != RT_OK) return r;
  hipError_t e = launch_build_lut(ctx->geo, make_bufs(nullptr, params, out), (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "build_lut");
}

rt_status rt_apply(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_lut_buf* lut,
                   const rt_stats_buf* whole_out, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_frames(ctx, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK) r = check_lut(lut);
  if (r == RT_OK && whole_out) r = check_stats(whole_out, false, true);
  if (r != RT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const FramePtrs fp = make_ptrs(ctx, frames, out_frames);
  const Bufs b = make_bufs(whole_out, nullptr, lut);
  if (whole_out) return whole_pass(ctx, ctx->geo, fp, b, true, true, st);
  hipError_t e = timed_apply(ctx, ctx->geo, fp, b, true, false, st);
  return e == hipSuccess ? RT_OK : hip_fail(e, "apply");
}

rt_status rt_apply_sets(rt_ctx* ctx, int32_t n, const void* const* frames, void* const* out_frames,
                        const rt_lut_buf* luts, const rt_stats_buf* wholes, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (n < 1 || n > kSetsMax) return fail(RT_EINVAL, "n %d outside 1..%d", n, kSetsMax);
  if (ctx->n_cams > kSetCams)
    return fail(RT_EUNSUPPORTED, "applies of several frame-sets take rigs of at most %d cameras (this one has %d)",
                kSetCams, ctx->n_cams);
  if (!frames || !out_frames || !luts || !wholes) return fail(RT_EINVAL, "frames, out_frames, luts or wholes is NULL");
  const int K = ctx->n_cams;
  rt_status r = RT_OK;
  for (int i = 0; r == RT_OK && i < n; ++i) {
    r = check_frames(ctx, frames + (int64_t)i * K, "frames");
    if (r == RT_OK) r = check_frames(ctx, (const void* const*)(out_frames + (int64_t)i * K), "out_frames");
    if (r == RT_OK) r = check_lut(&luts[i]);
    if (r == RT_OK) r = check_stats(&wholes[i], false, true);
  }
  if (r != RT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  SetPtrs sp;
  memset(&sp, 0, sizeof sp);
  sp.n_sets = n;
  hipError_t e = hipSuccess;
  for (int i = 0; e == hipSuccess && i < n; ++i) {
    const FramePtrs fp = make_ptrs(ctx, frames + (int64_t)i * K, out_frames + (int64_t)i * K);
    for (int k = 0; k < K; ++k) {
      sp.f[i].in[k] = fp.in[k];
      sp.f[i].out[k] = fp.out[k];
    }
    sp.b[i] = SetBufs{wholes[i].whole_hist, wholes[i].whole_sums, luts[i].lut8, luts[i].q16, luts[i].weights};
    e = launch_zero_whole(ctx->geo, make_bufs(&wholes[i], nullptr, nullptr), st);
  }
  if (e == hipSuccess) e = timed_apply_sets(ctx, ctx->geo, sp, st);
  return e == hipSuccess ? RT_OK : hip_fail(e, "apply of several frame-sets");
}

// The frame-set sequence over the cameras in `active`: band statistics,
// estimate + tables + clearing of the whole-frame statistics, apply.
static rt_status frameset_masked(rt_ctx* ctx, uint64_t active, const void* const* frames, void* const* out_frames,
                                 const rt_stats_buf* stats, const rt_params_buf* state, const rt_lut_buf* lut,
                                 void* stream) {
  rt_status r = check_frames_masked(ctx, active, frames, "frames");
  if (r == RT_OK) r = check_frames_masked(ctx, active, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK) r = check_stats(stats, true, true);
  if (r == RT_OK) r = check_params(state);
  if (r == RT_OK) r = check_lut(lut);
  if (r != RT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  Geo g = ctx->geo;
  g.active = active;
  const FramePtrs fp = make_ptrs_masked(ctx, frames, out_frames, active);
  const Bufs b = make_bufs(stats, state, lut);
  const hipError_t e = launch_band_estimate(g, fp, b, st);
  if (e != hipSuccess) return hip_fail(e, "band statistics, estimate and tables");
  return whole_pass(ctx, g, fp, b, true, false, st);
}

rt_status rt_frameset(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_stats_buf* stats,
                      const rt_params_buf* state, const rt_lut_buf* lut, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  return frameset_masked(ctx, ctx->geo.active, frames, out_frames, stats, state, lut, stream);
}

rt_status rt_frameset_batch(rt_ctx* ctx, uint64_t active, const void* const* frames, void* const* out_frames,
                            const rt_stats_buf* stats, const rt_params_buf* state, const rt_lut_buf* lut,
                            void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_active(ctx, active);
  if (r != RT_OK) return r;
  return frameset_masked(ctx, active, frames, out_frames, stats, state, lut, stream);
}

rt_status rt_frameset_ahead(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_lut_buf* lut,
                            const rt_stats_buf* whole, const void* const* next_frames, const rt_lut_buf* next_lut,
                            const rt_stats_buf* next_whole, const rt_stats_buf* bands, const rt_params_buf* state,
                            void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  const bool apply = frames != nullptr, est = next_frames != nullptr;
  if (!apply && !est) return fail(RT_EINVAL, "frames and next_frames are both NULL");
  rt_status r = RT_OK;
  if (apply) {
    r = check_frames(ctx, frames, "frames");
    if (r == RT_OK) r = check_frames(ctx, (const void* const*)out_frames, "out_frames");
    if (r == RT_OK) r = check_lut(lut);
    if (r == RT_OK) r = check_stats(whole, false, true);
  }
  if (est && r == RT_OK) {
    r = check_frames(ctx, next_frames, "next_frames");
    if (r == RT_OK) r = check_lut(next_lut);
    if (r == RT_OK) r = check_stats(next_whole, false, true);
    if (r == RT_OK) r = check_stats(bands, true, false);
    if (r == RT_OK) r = check_params(state);
  }
  if (r != RT_OK) return r;
  if (apply && est) {
    if (next_lut->lut8 == lut->lut8 || next_lut->q16 == lut->q16 || next_lut->weights == lut->weights)
      return fail(RT_EINVAL, "next_lut must be distinct from lut");
    if (next_whole->whole_hist == whole->whole_hist || next_whole->whole_sums == whole->whole_sums)
      return fail(RT_EINVAL, "next_whole must be distinct from whole");
  }
  FramePtrs fa, fe;
  Bufs ba, be;
  if (apply) {
    fa = make_ptrs(ctx, frames, out_frames);
    ba = make_bufs(whole, nullptr, lut);
  }
  if (est) {
    fe = make_ptrs(ctx, next_frames, nullptr);
    be = make_bufs(next_whole, state, next_lut);
    be.band_hist = bands->band_hist;
    be.band_sums = bands->band_sums;
  }
  const hipError_t e = launch_frameset_ahead(ctx->geo, apply ? &fa : nullptr, apply ? ba : be, est ? &fe : nullptr,
                                             est ? be : ba, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "look-ahead frame-set");
  return RT_OK;
}

rt_status rt_ctx_set_active(rt_ctx* ctx, uint64_t active) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_active(ctx, active);
  if (r == RT_OK) ctx->geo.active = active;
  return r;
}

rt_status rt_ctx_check(rt_ctx* ctx) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "device check");
  return RT_OK;
}

rt_status rt_ctx_tune(rt_ctx* ctx, int32_t tile_rows, int32_t grid) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (tile_rows < 1 || tile_rows > 4096) return fail(RT_EINVAL, "tile_rows %d outside 1..4096", tile_rows);
  if (grid < 0 || grid > kMaxApplyGrid) return fail(RT_EINVAL, "grid %d outside 0..%d", grid, kMaxApplyGrid);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  if (tile_rows == ctx->tile_rows && grid == ctx->grid) return RT_OK;
  return build_tables(ctx, tile_rows, grid);
}

// ---------------------------------------------------------------------------
// Object removal with the smoothing fallback (see ringcorr.h).
// ---------------------------------------------------------------------------
static rt_status check_removal(const rt_removal_opts* ro) {
  if (!ro) return fail(RT_EINVAL, "removal options are NULL");
  if (ro->tau < 0 || ro->tau > 255) return fail(RT_EINVAL, "tau %d outside 0..255", ro->tau);
  if (!(ro->min_kept >= 0.0 && ro->min_kept <= 1.0)) return fail(RT_EINVAL, "min_kept must lie in [0, 1]");
  return RT_OK;
}

static Removal make_removal(const rt_removal_opts* ro, uint64_t* kept_sums, uint8_t* method, bool has_prev) {
  Removal rm;
  memset(&rm, 0, sizeof rm);
  rm.kept_sums = kept_sums;
  rm.method = method;
  rm.tau = ro->tau;
  rm.has_prev = has_prev ? 1 : 0;
  rm.min_kept = ro->min_kept;
  return rm;
}

static PrevPtrs make_prev(const rt_ctx* ctx, const void* const* prev, uint64_t active) {
  PrevPtrs pp;
  memset(&pp, 0, sizeof pp);
  for (int k = 0; prev && k < ctx->n_cams; ++k)
    if ((active >> k) & 1ull) pp.in[k] = (const uint8_t*)prev[k];
  return pp;
}

rt_status rt_motion_stats(rt_ctx* ctx, const void* const* frames, const void* const* prev_frames,
                          const rt_removal_opts* ro, const rt_stats_buf* out, uint64_t* kept_sums, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_frames(ctx, frames, "frames");
  if (r == RT_OK && prev_frames) r = check_frames(ctx, prev_frames, "prev_frames");
  if (r == RT_OK) r = check_removal(ro);
  if (r == RT_OK) r = check_stats(out, true, false);
  if (r == RT_OK) r = check_ptr(kept_sums, 8, "kept_sums");
  if (r != RT_OK) return r;
  const FramePtrs fp = make_ptrs(ctx, frames, nullptr);
  const PrevPtrs pp = make_prev(ctx, prev_frames, ctx->geo.active);
  const Removal rm = make_removal(ro, kept_sums, nullptr, prev_frames != nullptr);
  hipError_t e = launch_motion_stats(ctx->geo, fp, pp, make_bufs(out, nullptr, nullptr), rm, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "motion statistics");
}

rt_status rt_estimate_removal(rt_ctx* ctx, const rt_stats_buf* stats, const uint64_t* kept_sums,
                              const rt_removal_opts* ro, const rt_params_buf* state, uint8_t* method, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (ctx->opts.fit != RT_FIT_MOMENTS) return fail(RT_EUNSUPPORTED, "object removal fits the moments only");
  rt_status r = check_stats(stats, true, false);
  if (r == RT_OK) r = check_removal(ro);
  if (r == RT_OK) r = check_ptr(kept_sums, 8, "kept_sums");
  if (r == RT_OK) r = check_params(state);
  if (r != RT_OK) return r;
  const Removal rm = make_removal(ro, const_cast<uint64_t*>(kept_sums), method, true);
  hipError_t e = launch_estimate_removal(ctx->geo, make_bufs(stats, state, nullptr), rm, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "removal estimate");
}

rt_status rt_frameset_removal(rt_ctx* ctx, const void* const* frames, const void* const* prev_frames,
                              void* const* out_frames, const rt_removal_opts* ro, const rt_stats_buf* stats,
                              uint64_t* kept_sums, const rt_params_buf* state, const rt_lut_buf* lut,
                              uint8_t* method, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (ctx->opts.fit != RT_FIT_MOMENTS) return fail(RT_EUNSUPPORTED, "object removal fits the moments only");
  const uint64_t active = ctx->geo.active;
  rt_status r = check_frames_masked(ctx, active, frames, "frames");
  if (r == RT_OK && prev_frames) r = check_frames_masked(ctx, active, prev_frames, "prev_frames");
  if (r == RT_OK) r = check_frames_masked(ctx, active, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK) r = check_removal(ro);
  if (r == RT_OK) r = check_stats(stats, true, true);
  if (r == RT_OK) r = check_ptr(kept_sums, 8, "kept_sums");
  if (r == RT_OK) r = check_params(state);
  if (r == RT_OK) r = check_lut(lut);
  if (r != RT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const Geo& g = ctx->geo;
  const FramePtrs fp = make_ptrs_masked(ctx, frames, out_frames, active);
  const PrevPtrs pp = make_prev(ctx, prev_frames, active);
  const Removal rm = make_removal(ro, kept_sums, method, prev_frames != nullptr);
  const Bufs b = make_bufs(stats, state, lut);
  const hipError_t e = launch_band_estimate_removal(g, fp, pp, b, rm, st);
  if (e != hipSuccess) return hip_fail(e, "band statistics with object removal, estimate and tables");
  return whole_pass(ctx, g, fp, b, true, false, st);
}

rt_status rt_graph_create(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_lut_buf* lut,
                          const rt_stats_buf* whole, const void* const* next_frames, const rt_lut_buf* next_lut,
                          const rt_stats_buf* bands, const rt_params_buf* state, rt_graph** out) {
  if (!out) return fail(RT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  const bool pipelined = next_frames != nullptr;
  rt_status r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_frames(ctx, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK) r = check_lut(lut);
  if (r == RT_OK) r = check_stats(whole, false, true);
  if (r == RT_OK) r = check_stats(bands, true, false);
  if (r == RT_OK) r = check_params(state);
  if (r == RT_OK && pipelined) r = check_frames(ctx, next_frames, "next_frames");
  if (r == RT_OK && pipelined) r = check_lut(next_lut);
  if (r != RT_OK) return r;
  if (pipelined && next_lut->lut8 == lut->lut8) return fail(RT_EINVAL, "next_lut must be distinct from lut");

  rt_graph* g = new (std::nothrow) rt_graph();
  if (!g) return fail(RT_ENOMEM, "host allocation failed");
  g->ctx = ctx;
  g->generation = ctx->generation;
  hipStream_t s0 = nullptr, s1 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s0, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s1, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_join, hipEventDisableTiming);
  bool begun = false;
  if (e == hipSuccess) e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    begun = true;
    ctx->capturing = true;
    const FramePtrs fp = make_ptrs(ctx, frames, out_frames);
    Bufs ba = make_bufs(whole, state, lut);          // apply branch
    ba.band_hist = bands->band_hist;
    ba.band_sums = bands->band_sums;
    if (!pipelined) {
      // bands -> estimate + tables (+ clearing the whole-frame statistics) -> apply -> reduction
      e = launch_band_estimate(ctx->geo, fp, ba, s0);
      if (e == hipSuccess) e = launch_apply(ctx->geo, fp, ba, true, true, s0);
    } else {
      // Branch E: statistics, estimate and tables of the next frame-set.
      // Branch A: apply of this frame-set with the tables estimated one step earlier.
      const FramePtrs fn = make_ptrs(ctx, next_frames, nullptr);
      Bufs be = make_bufs(nullptr, state, next_lut);
      be.band_hist = bands->band_hist;
      be.band_sums = bands->band_sums;
      e = hipEventRecord(ev_fork, s0);
      if (e == hipSuccess) e = hipStreamWaitEvent(s1, ev_fork, 0);
      if (e == hipSuccess) e = launch_band_estimate(ctx->geo, fn, be, s1);
      if (e == hipSuccess) e = launch_zero_whole(ctx->geo, ba, s0);
      if (e == hipSuccess) e = launch_apply(ctx->geo, fp, ba, true, true, s0);
      if (e == hipSuccess) e = hipEventRecord(ev_join, s1);
      if (e == hipSuccess) e = hipStreamWaitEvent(s0, ev_join, 0);
    }
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s0, &graph);
    if (e == hipSuccess) e = e2;
    g->graph = graph;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  g->pipelined = pipelined;
  if (e == hipSuccess) {
    // The nodes that rt_graph_set_frames rebinds: the band-statistics
    // kernel and the apply, each accepted only if its second argument holds
    // exactly the frame pointers it was captured with.
    const FramePtrs fp = make_ptrs(ctx, frames, out_frames);
    const FramePtrs fn = pipelined ? make_ptrs(ctx, next_frames, nullptr) : fp;
    const void* k_est = band_estimate_kernel(ctx->geo);
    const void* k_app = apply_kernel(ctx->geo, true, true);
    size_t n = 0;
    if (hipGraphGetNodes(g->graph, nullptr, &n) == hipSuccess && n > 0) {
      std::vector<hipGraphNode_t> nodes(n);
      if (hipGraphGetNodes(g->graph, nodes.data(), &n) == hipSuccess) {
        for (size_t i = 0; i < n; ++i) {
          hipGraphNodeType t;
          hipKernelNodeParams kp;
          if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
          if (hipGraphKernelNodeGetParams(nodes[i], &kp) != hipSuccess || !kp.kernelParams) continue;
          const bool est = kp.func == k_est, app = kp.func == k_app;
          if (!est && !app) continue;
          const FramePtrs& want = est && pipelined ? fn : fp;
          if (!kp.kernelParams[1] || memcmp(kp.kernelParams[1], &want, sizeof(FramePtrs)) != 0) continue;
          g->frame_nodes.push_back({nodes[i], est && pipelined});
        }
      }
    }
    if (g->frame_nodes.size() != 2) g->frame_nodes.clear();
  }
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (s1) (void)hipStreamDestroy(s1);
  if (s0) (void)hipStreamDestroy(s0);
  if (e != hipSuccess) {
    (void)begun;
    rt_graph_destroy(g);
    return hip_fail(e, "capturing the frame-set graph");
  }
  *out = g;
  return RT_OK;
}

rt_status rt_graph_set_frames(rt_graph* g, const void* const* frames, void* const* out_frames,
                              const void* const* next_frames) {
  if (!g || !g->exec) return fail(RT_EINVAL, "graph is NULL");
  rt_ctx* ctx = g->ctx;
  if (g->generation != ctx->generation)
    return fail(RT_ESTATE, "the context's tables were rebuilt after this graph was captured; capture it again");
  if (g->pipelined != (next_frames != nullptr))
    return fail(RT_EINVAL, g->pipelined ? "a two-branch graph needs next_frames" : "next_frames given for a one-branch graph");
  rt_status r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_frames(ctx, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK && next_frames) r = check_frames(ctx, next_frames, "next_frames");
  if (r != RT_OK) return r;
  if (g->frame_nodes.empty())
    return fail(RT_EUNSUPPORTED, "the graph's frame-pointer arguments were not found among its nodes");
  FramePtrs fp = make_ptrs(ctx, frames, out_frames);
  FramePtrs fn = next_frames ? make_ptrs(ctx, next_frames, nullptr) : fp;
  for (const auto& f : g->frame_nodes) {
    hipKernelNodeParams kp;
    hipError_t e = hipGraphKernelNodeGetParams(f.node, &kp);
    if (e != hipSuccess) return hip_fail(e, "reading a graph node");
    void* args[3] = {kp.kernelParams[0], f.next ? (void*)&fn : (void*)&fp, kp.kernelParams[2]};
    kp.kernelParams = args;
    kp.extra = nullptr;
    e = hipGraphExecKernelNodeSetParams(g->exec, f.node, &kp);
    if (e != hipSuccess) return hip_fail(e, "rebinding the graph's frames");
  }
  return RT_OK;
}

rt_status rt_graph_launch(rt_graph* g, void* stream) {
  if (!g || !g->exec) return fail(RT_EINVAL, "graph is NULL");
  if (g->generation != g->ctx->generation)
    return fail(RT_ESTATE, "the context's tables were rebuilt after this graph was captured; capture it again");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "graph launch");
}

rt_status rt_graph_destroy(rt_graph* g) {
  if (!g) return RT_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return RT_OK;
}

// ---------------------------------------------------------------------------
// Frame-set pipeline (see ringcorr.h).
//
// Host cost decides the design: on this runtime a kernel launch costs the
// host about 1 us, an event record about 5 us and a stream wait on an event
// that has not completed yet about 12 us (on a completed one about 1 us).
// So the statistics and estimates are launched on stream E as frame-sets
// are submitted, and the applies are issued a group at a time: one record
// on E after the group's estimates, then per lane one wait, the lane's
// applies of the group and one record.  Slot reuse waits on the record that
// covers the slot's previous apply, skipped when the event has completed.
// ---------------------------------------------------------------------------
constexpr int kMaxLanes = 4;
constexpr int kGroupRing = 12;                   // a slot's last apply is at most depth + 1 groups old

struct rt_pipe {
  rt_ctx* ctx = nullptr;
  int depth = 2, lanes = 1, group = 1;
  hipStream_t s_est = nullptr;                   // band statistics, estimate, tables (in order)
  hipStream_t s_lane[kMaxLanes - 1] = {};        // lanes 1..; lane 0 is the caller's stream
  hipEvent_t ev_est[kGroupRing] = {};            // per group: its estimates done (on E)
  hipEvent_t ev_lane[kGroupRing][kMaxLanes] = {};  // per group and lane: the lane's applies done
  std::vector<int64_t> slot_group;               // group of the slot's last apply (-1: none)
  std::vector<int> slot_lane;                    // its lane
  int last_group[kMaxLanes] = {-1, -1, -1, -1};  // per lane: last group with an apply on it
  rt_stats_buf bands{};
  rt_params_buf state{};
  std::vector<rt_lut_buf> luts;
  std::vector<rt_stats_buf> wholes;
  struct Pending { FramePtrs fp; uint64_t active; hipEvent_t done; int slot; int lane; };
  std::vector<Pending> pending;                  // estimated, apply not yet issued
  hipStream_t caller = nullptr;                  // lane 0 of the pending applies
  int64_t submitted = 0, groups = 0;
  int warm = 0;                                  // frame-sets since creation or the last join (capped)
  int fuse = 0;                                  // 1: a group's applies in one launch, groups over the lanes
  // Object removal (rt_pipe_set_removal): the options and buffers, and each
  // camera's frame of its last submit, which the next one is compared with.
  bool removal = false;
  Removal rm{};
  const uint8_t* prev_in[RT_MAX_CAMS] = {};
};

// Fused form: the group's applies go to one lane (groups take the lanes in
// turn) as launches of up to kSetsMax frame-sets with one camera mask, so
// the host pays one wait and one record per group.
static hipError_t pipe_flush_fused(rt_pipe* p) {
  rt_ctx* ctx = p->ctx;
  const int g = (int)(p->groups % kGroupRing), l = (int)(p->groups % p->lanes);
  hipStream_t sl = l ? p->s_lane[l - 1] : p->caller;
  hipError_t e = hipEventRecord(p->ev_est[g], p->s_est);
  if (e == hipSuccess) e = hipStreamWaitEvent(sl, p->ev_est[g], 0);
  const size_t np = p->pending.size();
  for (size_t i = 0; e == hipSuccess && i < np;) {
    size_t n = 1;
    while (i + n < np && n < (size_t)kSetsMax && p->pending[i + n].active == p->pending[i].active) ++n;
    SetPtrs sp;
    memset(&sp, 0, sizeof sp);
    sp.n_sets = (int32_t)n;
    for (size_t m = 0; m < n; ++m) {
      const auto& q = p->pending[i + m];
      for (int k = 0; k < ctx->n_cams; ++k) {
        sp.f[m].in[k] = q.fp.in[k];
        sp.f[m].out[k] = q.fp.out[k];
      }
      sp.b[m] = SetBufs{p->wholes[q.slot].whole_hist, p->wholes[q.slot].whole_sums, p->luts[q.slot].lut8,
                        p->luts[q.slot].q16, p->luts[q.slot].weights};
    }
    Geo gg = ctx->geo;
    gg.active = p->pending[i].active;
    e = timed_apply_sets(ctx, gg, sp, sl);
    for (size_t m = 0; m < n; ++m) {
      const auto& q = p->pending[i + m];
      if (e == hipSuccess && q.done) e = hipEventRecord(q.done, sl);
      p->slot_group[q.slot] = p->groups;
      p->slot_lane[q.slot] = l;
    }
    i += n;
  }
  if (e == hipSuccess) e = hipEventRecord(p->ev_lane[g][l], sl);
  p->last_group[l] = g;
  p->pending.clear();
  ++p->groups;
  return e;
}

// Issues the pending applies as one group (see above).
static hipError_t pipe_flush(rt_pipe* p) {
  if (p->pending.empty()) return hipSuccess;
  if (p->fuse) return pipe_flush_fused(p);
  rt_ctx* ctx = p->ctx;
  const int g = (int)(p->groups % kGroupRing);
  hipError_t e = hipEventRecord(p->ev_est[g], p->s_est);
  bool used[kMaxLanes] = {};
  for (const auto& q : p->pending) used[q.lane] = true;
  for (int l = 0; e == hipSuccess && l < p->lanes; ++l) {
    if (!used[l]) continue;
    hipStream_t sl = l ? p->s_lane[l - 1] : p->caller;
    e = hipStreamWaitEvent(sl, p->ev_est[g], 0);
    for (size_t i = 0; e == hipSuccess && i < p->pending.size(); ++i) {
      const auto& q = p->pending[i];
      if (q.lane != l) continue;
      const Bufs ba = make_bufs(&p->wholes[q.slot], nullptr, &p->luts[q.slot]);
      Geo g = ctx->geo;
      g.active = q.active;
      e = timed_apply(ctx, g, q.fp, ba, true, true, sl);
      if (e == hipSuccess && q.done) e = hipEventRecord(q.done, sl);
      p->slot_group[q.slot] = p->groups;
      p->slot_lane[q.slot] = l;
    }
    if (e == hipSuccess) e = hipEventRecord(p->ev_lane[g][l], sl);
    p->last_group[l] = (int)g;
  }
  p->pending.clear();
  ++p->groups;
  return e;
}

rt_status rt_pipe_create_lanes(rt_ctx* ctx, int32_t depth, int32_t lanes, int32_t group, const rt_stats_buf* bands,
                               const rt_params_buf* state, const rt_lut_buf* luts, const rt_stats_buf* wholes,
                               rt_pipe** out) {
  if (!out) return fail(RT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (depth < 1 || depth > 8) return fail(RT_EINVAL, "depth %d outside 1..8", depth);
  if (lanes < 1 || lanes > kMaxLanes) return fail(RT_EINVAL, "lanes %d outside 1..%d", lanes, kMaxLanes);
  if (depth < lanes) return fail(RT_EINVAL, "depth %d below lanes %d", depth, lanes);
  if (group < 1 || group > depth) return fail(RT_EINVAL, "group %d outside 1..depth (%d)", group, depth);
  if (!luts || !wholes) return fail(RT_EINVAL, "luts or wholes is NULL");
  rt_status r = check_stats(bands, true, false);
  if (r == RT_OK) r = check_params(state);
  for (int i = 0; r == RT_OK && i < depth; ++i) r = check_lut(&luts[i]);
  for (int i = 0; r == RT_OK && i < depth; ++i) r = check_stats(&wholes[i], false, true);
  if (r != RT_OK) return r;
  rt_pipe* p = new (std::nothrow) rt_pipe();
  if (!p) return fail(RT_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->depth = depth;
  p->lanes = lanes;
  p->group = group;
  p->bands = *bands;
  p->state = *state;
  p->luts.assign(luts, luts + depth);
  p->wholes.assign(wholes, wholes + depth);
  p->slot_group.assign(depth, -1);
  p->slot_lane.assign(depth, 0);
  p->pending.reserve(group);
  hipError_t e = hipStreamCreateWithFlags(&p->s_est, hipStreamNonBlocking);
  for (int l = 0; e == hipSuccess && l < lanes - 1; ++l) e = hipStreamCreateWithFlags(&p->s_lane[l], hipStreamNonBlocking);
  for (int g = 0; e == hipSuccess && g < kGroupRing; ++g) {
    e = hipEventCreateWithFlags(&p->ev_est[g], hipEventDisableTiming);
    for (int l = 0; e == hipSuccess && l < lanes; ++l) e = hipEventCreateWithFlags(&p->ev_lane[g][l], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    rt_pipe_destroy(p);
    return hip_fail(e, "creating the pipeline streams and events");
  }
  *out = p;
  return RT_OK;
}

rt_status rt_pipe_set_fuse(rt_pipe* p, int32_t fuse) {
  if (!p) return fail(RT_EINVAL, "pipe is NULL");
  if (fuse != 0 && fuse != 1) return fail(RT_EINVAL, "fuse %d is not 0 or 1", fuse);
  if (fuse && p->ctx->n_cams > kSetCams)
    return fail(RT_EUNSUPPORTED, "fused applies take rigs of at most %d cameras (this one has %d)", kSetCams,
                p->ctx->n_cams);
  const hipError_t e = pipe_flush(p);
  if (e != hipSuccess) return hip_fail(e, "pipeline flush");
  p->fuse = fuse;
  return RT_OK;
}

rt_status rt_pipe_set_removal(rt_pipe* p, const rt_removal_opts* ro, uint64_t* kept_sums, uint8_t* method) {
  if (!p) return fail(RT_EINVAL, "pipe is NULL");
  if (!ro) {
    p->removal = false;
    return RT_OK;
  }
  if (p->ctx->opts.fit != RT_FIT_MOMENTS) return fail(RT_EUNSUPPORTED, "object removal fits the moments only");
  rt_status r = check_removal(ro);
  if (r == RT_OK) r = check_ptr(kept_sums, 8, "kept_sums");
  if (r != RT_OK) return r;
  p->rm = make_removal(ro, kept_sums, method, false);
  memset(p->prev_in, 0, sizeof p->prev_in);
  p->removal = true;
  return RT_OK;
}

rt_status rt_pipe_create(rt_ctx* ctx, int32_t depth, const rt_stats_buf* bands, const rt_params_buf* state,
                         const rt_lut_buf* luts, const rt_stats_buf* wholes, rt_pipe** out) {
  return rt_pipe_create_lanes(ctx, depth, 1, 1, bands, state, luts, wholes, out);
}

static rt_status pipe_submit(rt_pipe* p, uint64_t active, const void* const* frames, void* const* out_frames,
                             void* stream, void* ready_event, void* done_event, int32_t* slot_out) {
  rt_ctx* ctx = p->ctx;
  rt_status r = check_frames_masked(ctx, active, frames, "frames");
  if (r == RT_OK) r = check_frames_masked(ctx, active, (const void* const*)out_frames, "out_frames");
  if (r != RT_OK) return r;
  if (done_event && p->group != 1) return fail(RT_EINVAL, "done_event needs a pipeline with group 1");
  // With object removal the next submit's statistics read this frame-set's
  // inputs, unordered with respect to this apply: it must not overwrite them.
  if (p->removal)
    for (int k = 0; k < ctx->n_cams; ++k)
      if (((active >> k) & 1ull) && frames[k] == out_frames[k])
        return fail(RT_EINVAL, "camera %d: an in-place frame-set cannot be pipelined with object removal", k);
  const int slot = (int)(p->submitted % p->depth);
  hipError_t e = hipSuccess;
  // The slot's previous apply may still be pending: issue it first.
  for (const auto& q : p->pending)
    if (q.slot == slot) { e = pipe_flush(p); break; }
  // Pending applies run on the stream they were submitted on.
  if (e == hipSuccess && !p->pending.empty() && p->caller != (hipStream_t)stream) e = pipe_flush(p);
  p->caller = (hipStream_t)stream;
  Geo g = ctx->geo;
  g.active = active;
  const FramePtrs fp = make_ptrs_masked(ctx, frames, out_frames, active);
  Bufs be = make_bufs(&p->bands, &p->state, &p->luts[slot]);
  be.whole_hist = p->wholes[slot].whole_hist;    // cleared by the estimate kernel
  be.whole_sums = p->wholes[slot].whole_sums;
  // Stream E, in submission order: after the frames are ready (ready_event)
  // and after the apply that last used this slot, the band statistics,
  // estimate and tables.  Band statistics and estimator state are single
  // buffers, so their order on E gives the results of consecutive frame-sets.
  if (e == hipSuccess && ready_event) e = hipStreamWaitEvent(p->s_est, (hipEvent_t)ready_event, 0);
  if (e == hipSuccess && p->slot_group[slot] >= 0) {
    hipEvent_t prev = p->ev_lane[p->slot_group[slot] % kGroupRing][p->slot_lane[slot]];
    const hipError_t q = hipEventQuery(prev);
    if (q == hipErrorNotReady) e = hipStreamWaitEvent(p->s_est, prev, 0);
    else if (q != hipSuccess) e = q;
  }
  if (e == hipSuccess && p->removal) {
    // Against each active camera's frame of its last submit; if one has
    // none yet, nothing moves in this frame-set.
    PrevPtrs pp;
    memset(&pp, 0, sizeof pp);
    bool has_prev = true;
    for (int k = 0; k < ctx->n_cams; ++k)
      if ((active >> k) & 1ull) {
        pp.in[k] = p->prev_in[k];
        has_prev = has_prev && p->prev_in[k] != nullptr;
      }
    if (!has_prev) memset(&pp, 0, sizeof pp);
    Removal rm = p->rm;
    rm.has_prev = has_prev ? 1 : 0;
    e = launch_band_estimate_removal(g, fp, pp, be, rm, p->s_est);
    if (e == hipSuccess)
      for (int k = 0; k < ctx->n_cams; ++k)
        if ((active >> k) & 1ull) p->prev_in[k] = fp.in[k];
  } else if (e == hipSuccess) {
    e = launch_band_estimate(g, fp, be, p->s_est);
  }
  if (e == hipSuccess) {
    p->pending.push_back({fp, active, (hipEvent_t)done_event, slot, (int)(p->submitted % p->lanes)});
    // An idle pipeline issues its first `lanes` applies one at a time, so
    // that they do not wait for a full group of estimates.
    if ((int)p->pending.size() == p->group || p->warm < p->lanes) e = pipe_flush(p);
    if (p->warm < p->lanes) ++p->warm;
  }
  if (e != hipSuccess) return hip_fail(e, "pipeline submit");
  if (slot_out) *slot_out = slot;
  ++p->submitted;
  return RT_OK;
}

rt_status rt_pipe_submit(rt_pipe* p, const void* const* frames, void* const* out_frames, void* stream,
                         void* ready_event, int32_t* slot_out) {
  if (!p) return fail(RT_EINVAL, "pipe is NULL");
  return pipe_submit(p, p->ctx->geo.active, frames, out_frames, stream, ready_event, nullptr, slot_out);
}

rt_status rt_pipe_submit_batch(rt_pipe* p, uint64_t active, const void* const* frames, void* const* out_frames,
                               void* stream, void* ready_event, void* done_event, int32_t* slot_out) {
  if (!p) return fail(RT_EINVAL, "pipe is NULL");
  const rt_status r = check_active(p->ctx, active);
  if (r != RT_OK) return r;
  return pipe_submit(p, active, frames, out_frames, stream, ready_event, done_event, slot_out);
}

rt_status rt_pipe_submit_n(rt_pipe* p, int32_t n, const void* const* frames, void* const* out_frames, void* stream,
                           int32_t* slots_out, int32_t* n_done) {
  if (n_done) *n_done = 0;
  if (!p) return fail(RT_EINVAL, "pipe is NULL");
  if (n < 0) return fail(RT_EINVAL, "n %d < 0", n);
  if (n > 0 && (!frames || !out_frames)) return fail(RT_EINVAL, "frames or out_frames is NULL");
  const int K = p->ctx->n_cams;
  for (int i = 0; i < n; ++i) {
    int32_t slot = 0;
    const rt_status r = pipe_submit(p, p->ctx->geo.active, frames + (int64_t)i * K, out_frames + (int64_t)i * K,
                                    stream, nullptr, nullptr, &slot);
    if (r != RT_OK) return r;
    if (slots_out) slots_out[i] = slot;
    if (n_done) *n_done = i + 1;
  }
  return RT_OK;
}

rt_status rt_pipe_join(rt_pipe* p, void* stream) {
  if (!p) return fail(RT_EINVAL, "pipe is NULL");
  hipError_t e = pipe_flush(p);
  p->warm = 0;
  for (int l = 0; e == hipSuccess && l < p->lanes; ++l)
    if (p->last_group[l] >= 0) e = hipStreamWaitEvent((hipStream_t)stream, p->ev_lane[p->last_group[l]][l], 0);
  return e == hipSuccess ? RT_OK : hip_fail(e, "pipeline join");
}

rt_status rt_pipe_destroy(rt_pipe* p) {
  if (!p) return RT_OK;
  (void)pipe_flush(p);
  if (p->s_est) (void)hipStreamSynchronize(p->s_est);
  for (int l = 0; l < p->lanes; ++l)
    if (p->last_group[l] >= 0) (void)hipEventSynchronize(p->ev_lane[p->last_group[l]][l]);
  for (int g = 0; g < kGroupRing; ++g) {
    if (p->ev_est[g]) (void)hipEventDestroy(p->ev_est[g]);
    for (int l = 0; l < kMaxLanes; ++l)
      if (p->ev_lane[g][l]) (void)hipEventDestroy(p->ev_lane[g][l]);
  }
  for (int l = 0; l < kMaxLanes - 1; ++l)
    if (p->s_lane[l]) (void)hipStreamDestroy(p->s_lane[l]);
  if (p->s_est) (void)hipStreamDestroy(p->s_est);
  delete p;
  return RT_OK;
}

// ---------------------------------------------------------------------------
// Learned surrogate.
// ---------------------------------------------------------------------------
static rt_status check_mlp(const rt_mlp* m, const char* name) {
  if (!m) return fail(RT_EINVAL, "%s is NULL", name);
  const float* p[6] = {m->w1, m->b1, m->w2, m->b2, m->w3, m->b3};
  for (int i = 0; i < 6; ++i)
    if (!p[i] || !aligned(p[i], 4)) return fail(RT_EINVAL, "%s tensor %d is NULL or misaligned", name, i);
  return RT_OK;
}

rt_status rt_surrogate_features(rt_ctx* ctx, const rt_stats_buf* stats, float* X, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (!stats) return fail(RT_EINVAL, "stats buffer struct is NULL");
  rt_status r = check_ptr(stats->band_hist, 4, "band_hist");
  if (r == RT_OK) r = check_ptr(stats->whole_hist, 4, "whole_hist");
  if (r == RT_OK) r = check_ptr(X, 4, "X");
  if (r != RT_OK) return r;
  hipError_t e = launch_features(ctx->geo, stats->band_hist, stats->whole_hist, X, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "surrogate features");
}

rt_status rt_estimate_new(rt_ctx* ctx, const rt_stats_buf* stats, double* p_new, int32_t* status, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (ctx->opts.fit != RT_FIT_MOMENTS) return fail(RT_EUNSUPPORTED, "the surrogate's plain estimate fits the moments only");
  if (!stats) return fail(RT_EINVAL, "stats buffer struct is NULL");
  rt_status r = check_ptr(stats->band_sums, 8, "band_sums");
  if (r == RT_OK) r = check_ptr(p_new, 8, "p_new");
  if (r == RT_OK) r = check_ptr(status, 4, "status");
  if (r != RT_OK) return r;
  hipError_t e = launch_estimate_new(ctx->geo, stats->band_sums, p_new, status, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "plain estimate");
}

rt_status rt_surrogate_targets(rt_ctx* ctx, const double* p_new, const int32_t* status, float* T, uint8_t* mask,
                               void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_ptr(p_new, 8, "p_new");
  if (r == RT_OK) r = check_ptr(status, 4, "status");
  if (r == RT_OK) r = check_ptr(T, 4, "T");
  if (r == RT_OK) r = check_ptr(mask, 1, "mask");
  if (r != RT_OK) return r;
  hipError_t e = launch_targets(ctx->geo, p_new, status, T, mask, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "surrogate targets");
}

rt_status rt_surrogate_select(rt_ctx* ctx, const float* Y, const double* p_new, const int32_t* status, float tol,
                              const rt_params_buf* state, uint8_t* used, float* residual, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  rt_status r = check_ptr(Y, 4, "Y");
  if (r == RT_OK) r = check_ptr(p_new, 8, "p_new");
  if (r == RT_OK) r = check_ptr(status, 4, "status");
  if (r == RT_OK) r = check_params(state);
  if (r == RT_OK) r = check_ptr(used, 1, "used");
  if (r == RT_OK) r = check_ptr(residual, 4, "residual");
  if (r != RT_OK) return r;
  if (!(tol >= 0.0f)) return fail(RT_EINVAL, "tol must be >= 0");
  hipError_t e = launch_select(ctx->geo, Y, p_new, status, tol, state->params, state->valid, used, residual,
                               (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "surrogate select");
}

static void mlp_ptrs(const rt_mlp* m, float** out) {
  out[0] = m->w1; out[1] = m->b1; out[2] = m->w2; out[3] = m->b2; out[4] = m->w3; out[5] = m->b3;
}

// Launches of rt_surrogate_frameset once its arguments are validated; the
// workspace regions are device pointers of the caller's or of the static
// workspace below.
static rt_status surrogate_frameset_run(rt_ctx* ctx, const rt_mlp* w, float tol, const void* const* frames,
                                        void* const* out_frames, const rt_stats_buf* stats,
                                        const uint32_t* whole_hist_prev, const rt_params_buf* state,
                                        const rt_lut_buf* lut, const rt_surrogate_work* work, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const Geo& g = ctx->geo;
  const FramePtrs fp = make_ptrs_masked(ctx, frames, out_frames, g.active);
  const Bufs b = make_bufs(stats, state, lut);
  hipError_t e = launch_band_stats(g, fp, b, st);
  if (e != hipSuccess) return hip_fail(e, "band statistics");
  e = launch_features_new(g, b.band_hist, b.band_sums, whole_hist_prev, work->X, work->p_new, work->status, st);
  if (e != hipSuccess) return hip_fail(e, "surrogate features and plain estimate");
  float* wp[6];
  mlp_ptrs(w, wp);
  e = mlp_hidden(wp, work->X, g.n_cams * 2 * g.n_blocks, work->H1, work->H2, st);
  if (e != hipSuccess) return hip_fail(e, "mlp hidden layers");
  e = launch_select_lut(g, work->H2, w->w3, w->b3, work->Y, work->p_new, work->status, tol, b, work->used,
                        work->residual, st);
  if (e != hipSuccess) return hip_fail(e, "surrogate choice and tables");
  return whole_pass(ctx, g, fp, b, true, false, st);
}

// Arguments of rt_surrogate_frameset other than the workspace.
static rt_status check_surrogate_frameset(rt_ctx* ctx, const rt_mlp* w, float tol, const void* const* frames,
                                          void* const* out_frames, const rt_stats_buf* stats,
                                          const uint32_t* whole_hist_prev, const rt_params_buf* state,
                                          const rt_lut_buf* lut) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (ctx->opts.fit != RT_FIT_MOMENTS) return fail(RT_EUNSUPPORTED, "the surrogate's plain estimate fits the moments only");
  const uint64_t active = ctx->geo.active;
  rt_status r = check_mlp(w, "weights");
  if (r == RT_OK) r = check_frames_masked(ctx, active, frames, "frames");
  if (r == RT_OK) r = check_frames_masked(ctx, active, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK) r = check_stats(stats, true, true);
  if (r == RT_OK) r = check_ptr(whole_hist_prev, 4, "whole_hist_prev");
  if (r == RT_OK) r = check_params(state);
  if (r == RT_OK) r = check_lut(lut);
  if (r != RT_OK) return r;
  if (!(tol >= 0.0f)) return fail(RT_EINVAL, "tol must be >= 0");
  return RT_OK;
}

rt_status rt_surrogate_frameset(rt_ctx* ctx, const rt_mlp* w, float tol, const void* const* frames,
                                void* const* out_frames, const rt_stats_buf* stats, const uint32_t* whole_hist_prev,
                                const rt_params_buf* state, const rt_lut_buf* lut, const rt_surrogate_work* work,
                                void* stream) {
  rt_status r = check_surrogate_frameset(ctx, w, tol, frames, out_frames, stats, whole_hist_prev, state, lut);
  if (r != RT_OK) return r;
  if (!work) return fail(RT_EINVAL, "work struct is NULL");
  const void* fw[4] = {work->X, work->H1, work->H2, work->Y};
  for (int i = 0; i < 4; ++i)
    if ((r = check_ptr(fw[i], 4, "work activation")) != RT_OK) return r;
  if ((r = check_ptr(work->p_new, 8, "work p_new")) != RT_OK) return r;
  if ((r = check_ptr(work->status, 4, "work status")) != RT_OK) return r;
  if ((r = check_ptr(work->used, 1, "work used")) != RT_OK) return r;
  if ((r = check_ptr(work->residual, 4, "work residual")) != RT_OK) return r;
  return surrogate_frameset_run(ctx, w, tol, frames, out_frames, stats, whole_hist_prev, state, lut, work, stream);
}

// ---------------------------------------------------------------------------
// The workspace of rt_surrogate_frameset_static: a file-scope device array
// (every GPU the library runs on holds its own copy until the process ends),
// found through hipGetSymbolAddress once per device when the first context on
// that device is created.  Host code uses only the device address kept here,
// never the array's name.  Regions for kStaticUnits units, each 256-byte
// aligned: X f32 [U][576], H1 and H2 f32 [U][256], Y f32 [U][6], p_new f64
// [U][3][2], status i32 [U][3], used u8 [U], residual f32 [U].
namespace {
constexpr size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
constexpr size_t kStOffX = 0;
constexpr size_t kStOffH1 = kStOffX + align256((size_t)RT_STATIC_UNITS * kMlpIn * 4);
constexpr size_t kStOffH2 = kStOffH1 + align256((size_t)RT_STATIC_UNITS * kMlpHid * 4);
constexpr size_t kStOffY = kStOffH2 + align256((size_t)RT_STATIC_UNITS * kMlpHid * 4);
constexpr size_t kStOffP = kStOffY + align256((size_t)RT_STATIC_UNITS * kMlpOut * 4);
constexpr size_t kStOffS = kStOffP + align256((size_t)RT_STATIC_UNITS * 6 * 8);
constexpr size_t kStOffU = kStOffS + align256((size_t)RT_STATIC_UNITS * 3 * 4);
constexpr size_t kStOffR = kStOffU + align256((size_t)RT_STATIC_UNITS);
constexpr size_t kStaticBytes = kStOffR + align256((size_t)RT_STATIC_UNITS * 4);
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};        // device address of `scratch` on each device
hipError_t g_scratch_err[kMaxDevices] = {};   // result of the lookup (hipSuccess once found)
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// Looks the array up on `device` (the current device) once; later calls
// return the kept result.
static hipError_t static_scratch(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? p : nullptr;
    g_scratch_done[device] = true;
  }
  *out = g_scratch_ptr[device];
  return g_scratch_err[device];
}

rt_status rt_surrogate_frameset_static(rt_ctx* ctx, const rt_mlp* w, float tol, const void* const* frames,
                                       void* const* out_frames, const rt_stats_buf* stats,
                                       const uint32_t* whole_hist_prev, const rt_params_buf* state,
                                       const rt_lut_buf* lut, void* stream) {
  rt_status r = check_surrogate_frameset(ctx, w, tol, frames, out_frames, stats, whole_hist_prev, state, lut);
  if (r != RT_OK) return r;
  const int64_t units = (int64_t)ctx->n_cams * 2 * ctx->opts.n_blocks;
  if (units > RT_STATIC_UNITS)
    return fail(RT_EUNSUPPORTED, "%lld units (cameras x 2 x n_blocks) exceed the static workspace of %d units",
                (long long)units, RT_STATIC_UNITS);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev != ctx->device) return fail(RT_EINVAL, "the context lives on device %d, the current device is %d",
                                      ctx->device, dev);
  void* base = nullptr;
  e = static_scratch(dev, &base);
  if (e != hipSuccess || !base) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "static workspace");
  unsigned char* p = static_cast<unsigned char*>(base);
  rt_surrogate_work work;
  work.X = reinterpret_cast<float*>(p + kStOffX);
  work.H1 = reinterpret_cast<float*>(p + kStOffH1);
  work.H2 = reinterpret_cast<float*>(p + kStOffH2);
  work.Y = reinterpret_cast<float*>(p + kStOffY);
  work.p_new = reinterpret_cast<double*>(p + kStOffP);
  work.status = reinterpret_cast<int32_t*>(p + kStOffS);
  work.used = p + kStOffU;
  work.residual = reinterpret_cast<float*>(p + kStOffR);
  return surrogate_frameset_run(ctx, w, tol, frames, out_frames, stats, whole_hist_prev, state, lut, &work, stream);
}

rt_status rt_mlp_forward(const rt_mlp* w, const float* X, int32_t n, float* H1, float* H2, float* Y, void* stream) {
  rt_status r = check_mlp(w, "weights");
  if (r == RT_OK) r = check_ptr(X, 4, "X");
  if (r == RT_OK) r = check_ptr(H1, 4, "H1");
  if (r == RT_OK) r = check_ptr(H2, 4, "H2");
  if (r == RT_OK) r = check_ptr(Y, 4, "Y");
  if (r != RT_OK) return r;
  if (n < 0) return fail(RT_EINVAL, "n < 0");
  float* wp[6];
  mlp_ptrs(w, wp);
  hipError_t e = mlp_forward(wp, X, n, H1, H2, Y, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "mlp forward");
}

rt_status rt_mlp_backward(const rt_mlp* w, const float* X, const float* H1, const float* H2, const float* Y,
                          const float* T, int32_t n, const rt_mlp* grad, float* dY, float* dZ1, float* dZ2,
                          void* stream) {
  rt_status r = check_mlp(w, "weights");
  if (r == RT_OK) r = check_mlp(grad, "grad");
  const void* ps[8] = {X, H1, H2, Y, T, dY, dZ1, dZ2};
  for (int i = 0; r == RT_OK && i < 8; ++i) r = check_ptr(ps[i], 4, "activation or workspace");
  if (r != RT_OK) return r;
  if (n < 1) return fail(RT_EINVAL, "n < 1");
  float *wp[6], *gp[6];
  mlp_ptrs(w, wp);
  mlp_ptrs(grad, gp);
  hipError_t e = mlp_backward(wp, X, H1, H2, Y, T, n, gp, dY, dZ1, dZ2, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "mlp backward");
}

rt_status rt_mlp_adam(const rt_mlp* w, const rt_mlp* grad, const rt_mlp* m, const rt_mlp* v, int32_t step, float lr,
                      float beta1, float beta2, float eps, void* stream) {
  rt_status r = check_mlp(w, "weights");
  if (r == RT_OK) r = check_mlp(grad, "grad");
  if (r == RT_OK) r = check_mlp(m, "m");
  if (r == RT_OK) r = check_mlp(v, "v");
  if (r != RT_OK) return r;
  if (step < 1) return fail(RT_EINVAL, "step must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr > 0.0f))
    return fail(RT_EINVAL, "need 0 <= beta < 1, eps > 0, lr > 0");
  float *wp[6], *gp[6], *mp[6], *vp[6];
  mlp_ptrs(w, wp);
  mlp_ptrs(grad, gp);
  mlp_ptrs(m, mp);
  mlp_ptrs(v, vp);
  hipError_t e = mlp_adam(wp, gp, mp, vp, step, lr, beta1, beta2, eps, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "adam");
}

rt_status rt_mlp_mse(const float* Y, const float* T, int32_t n, float* out, void* stream) {
  rt_status r = check_ptr(Y, 4, "Y");
  if (r == RT_OK) r = check_ptr(T, 4, "T");
  if (r == RT_OK) r = check_ptr(out, 4, "out");
  if (r != RT_OK) return r;
  if (n < 1) return fail(RT_EINVAL, "n < 1");
  hipError_t e = mlp_mse(Y, T, n, out, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "mse");
}

rt_status rt_gather_rows(const float* src, int32_t row_len, const int32_t* idx, int32_t n, float* dst,
                         void* stream) {
  rt_status r = check_ptr(src, 4, "src");
  if (r == RT_OK) r = check_ptr(idx, 4, "idx");
  if (r == RT_OK) r = check_ptr(dst, 4, "dst");
  if (r != RT_OK) return r;
  if (row_len < 1 || n < 0) return fail(RT_EINVAL, "row_len < 1 or n < 0");
  hipError_t e = gather_rows(src, row_len, idx, n, dst, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "gather rows");
}

rt_status rt_mlp_train(const rt_mlp* w, const rt_mlp* grad, const rt_mlp* m, const rt_mlp* v, const float* X,
                       const float* T, int32_t n_rows, const int32_t* idx, int32_t batch, int32_t n_steps,
                       int32_t step0, float lr, float beta1, float beta2, float eps, const rt_mlp_work* work,
                       float* losses, void* stream) {
  rt_status r = check_mlp(w, "weights");
  if (r == RT_OK) r = check_mlp(grad, "grad");
  if (r == RT_OK) r = check_mlp(m, "m");
  if (r == RT_OK) r = check_mlp(v, "v");
  if (r == RT_OK) r = check_ptr(X, 4, "X");
  if (r == RT_OK) r = check_ptr(T, 4, "T");
  if (r == RT_OK) r = check_ptr(idx, 4, "idx");
  if (r == RT_OK) r = check_ptr(losses, 4, "losses");
  if (r == RT_OK && !work) r = fail(RT_EINVAL, "work is NULL");
  if (r == RT_OK) {
    const void* ws[8] = {work->xb, work->tb, work->h1, work->h2, work->y, work->dy, work->dz1, work->dz2};
    for (int i = 0; r == RT_OK && i < 8; ++i) r = check_ptr(ws[i], 4, "workspace");
  }
  if (r != RT_OK) return r;
  if (n_rows < 1 || batch < 1 || n_steps < 0) return fail(RT_EINVAL, "need n_rows >= 1, batch >= 1, n_steps >= 0");
  if (step0 < 1) return fail(RT_EINVAL, "step0 must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr > 0.0f))
    return fail(RT_EINVAL, "need 0 <= beta < 1, eps > 0, lr > 0");
  float *wp[6], *gp[6], *mp[6], *vp[6];
  mlp_ptrs(w, wp);
  mlp_ptrs(grad, gp);
  mlp_ptrs(m, mp);
  mlp_ptrs(v, vp);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int s = 0; e == hipSuccess && s < n_steps; ++s) {
    const int32_t* ix = idx + (int64_t)s * batch;
    // The per-step calls' sequence with the two gathers in one launch and the
    // loss gradient computed by the output layer (the same arithmetic).
    e = gather_rows2(X, kMlpIn, work->xb, T, kMlpOut, work->tb, ix, batch, st);
    if (e == hipSuccess) e = mlp_forward(wp, work->xb, batch, work->h1, work->h2, work->y, st, work->tb, work->dy);
    if (e == hipSuccess)
      e = mlp_backward(wp, work->xb, work->h1, work->h2, work->y, work->tb, batch, gp, work->dy, work->dz1,
                       work->dz2, st, true);
    if (e == hipSuccess) e = mlp_adam(wp, gp, mp, vp, step0 + s, lr, beta1, beta2, eps, st);
    if (e == hipSuccess) e = mlp_mse(work->y, work->tb, batch, losses + s, st);
  }
  return e == hipSuccess ? RT_OK : hip_fail(e, "mlp train");
}

rt_status rt_ctx_timing(rt_ctx* ctx, int32_t slots, int32_t every) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (slots < 0 || slots > 65536) return fail(RT_EINVAL, "slots %d outside 0..65536", slots);
  if (every < 1) return fail(RT_EINVAL, "every %d < 1", every);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  free_timing(ctx);
  ctx->timing_every = every;
  ctx->n_applies = 0;
  for (int i = 0; i < slots; ++i) {
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      free_timing(ctx);
      return hip_fail(e, "creating timing events");
    }
    ctx->ev_begin.push_back(a);
    ctx->ev_end.push_back(b);
  }
  ctx->timed_sets.assign(slots, 0);
  ctx->n_timing = slots;
  return RT_OK;
}

rt_status rt_ctx_apply_times(rt_ctx* ctx, float* ms, int32_t max_n, int32_t* n_out) {
  if (!ctx || !ms || !n_out || max_n < 0) return fail(RT_EINVAL, "ctx, ms or n_out is NULL, or max_n < 0");
  *n_out = 0;
  if (ctx->n_timing <= 0) return RT_OK;
  const int64_t avail = std::min<int64_t>(ctx->n_timed, ctx->n_timing);
  const int n = (int)std::min<int64_t>(avail, max_n);
  for (int i = 0; i < n; ++i) {
    const int slot = (int)((ctx->n_timed - n + i) % ctx->n_timing);
    hipError_t e = hipEventSynchronize(ctx->ev_end[slot]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], ctx->ev_begin[slot], ctx->ev_end[slot]);
    if (e != hipSuccess) return hip_fail(e, "reading timing events");
  }
  *n_out = n;
  return RT_OK;
}

rt_status rt_ctx_apply_sets(const rt_ctx* ctx, int32_t* sets, int32_t max_n, int32_t* n_out) {
  if (!ctx || !sets || !n_out || max_n < 0) return fail(RT_EINVAL, "ctx, sets or n_out is NULL, or max_n < 0");
  *n_out = 0;
  if (ctx->n_timing <= 0) return RT_OK;
  const int64_t avail = std::min<int64_t>(ctx->n_timed, ctx->n_timing);
  const int n = (int)std::min<int64_t>(avail, max_n);
  for (int i = 0; i < n; ++i) sets[i] = ctx->timed_sets[(size_t)((ctx->n_timed - n + i) % ctx->n_timing)];
  *n_out = n;
  return RT_OK;
}

// ---------------------------------------------------------------- cross-channel 3x3 maps

static rt_status check_cross_ctx(const rt_ctx* ctx) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  for (int k = 0; k < ctx->n_cams; ++k)
    if (ctx->cams[k].channels != 3 || ctx->cams[k].bit_depth != 8)
      return fail(RT_EUNSUPPORTED, "cross-channel maps need 8-bit RGB cameras (camera %d)", k);
  if (ctx->opts.vblend) return fail(RT_EUNSUPPORTED, "cross-channel maps are not blended between blocks");
  if (ctx->opts.fit != RT_FIT_MOMENTS) return fail(RT_EUNSUPPORTED, "cross-channel maps fit the moments only");
  return RT_OK;
}

static rt_status check_cross(const rt_cross_buf* x, bool cross, bool state, bool q3, bool weights) {
  if (!x) return fail(RT_EINVAL, "cross buffer struct is NULL");
  rt_status r = RT_OK;
  if (cross && (r = check_ptr(x->cross, 8, "cross")) != RT_OK) return r;
  if (state && (r = check_ptr(x->params3, 8, "params3")) != RT_OK) return r;
  if (state && (r = check_ptr(x->valid3, 1, "valid3")) != RT_OK) return r;
  if (q3 && (r = check_ptr(x->q3, 8, "q3")) != RT_OK) return r;
  if (weights && (r = check_ptr(x->weights, 2, "weights")) != RT_OK) return r;
  return RT_OK;
}

static CrossBufs make_cross(const rt_cross_buf* x) {
  return CrossBufs{x->cross, x->params3, x->valid3, x->q3, x->weights};
}

rt_status rt_cross_stats(rt_ctx* ctx, const void* const* frames, const rt_cross_buf* x, void* stream) {
  rt_status r = check_cross_ctx(ctx);
  if (r == RT_OK) r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_cross(x, true, false, false, false);
  if (r != RT_OK) return r;
  const hipError_t e = launch_cross_stats(ctx->geo, make_ptrs(ctx, frames, nullptr), make_cross(x), (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "cross statistics");
}

rt_status rt_estimate_cross(rt_ctx* ctx, const rt_stats_buf* stats, const rt_cross_buf* x, void* stream) {
  rt_status r = check_cross_ctx(ctx);
  if (r == RT_OK && !stats) r = fail(RT_EINVAL, "stats buffer struct is NULL");
  if (r == RT_OK) r = check_ptr(stats->band_sums, 8, "band_sums");
  if (r == RT_OK) r = check_cross(x, true, true, false, false);
  if (r != RT_OK) return r;
  const hipError_t e = launch_estimate_cross(ctx->geo, make_bufs(stats, nullptr, nullptr), make_cross(x),
                                             (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "cross-channel estimate");
}

rt_status rt_build_cross(rt_ctx* ctx, const rt_cross_buf* x, void* stream) {
  rt_status r = check_cross_ctx(ctx);
  if (r == RT_OK) r = check_cross(x, false, true, true, true);
  if (r != RT_OK) return r;
  const hipError_t e = launch_build_cross(ctx->geo, make_cross(x), (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "cross-channel maps");
}

rt_status rt_apply_cross(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_cross_buf* x,
                         const rt_stats_buf* whole_out, void* stream) {
  rt_status r = check_cross_ctx(ctx);
  if (r == RT_OK) r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_frames(ctx, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK) r = check_cross(x, false, false, true, true);
  if (r == RT_OK && whole_out) r = check_stats(whole_out, false, true);
  if (r != RT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const Bufs b = make_bufs(whole_out, nullptr, nullptr);
  hipError_t e = hipSuccess;
  if (whole_out) e = launch_zero_whole(ctx->geo, b, st);
  if (e == hipSuccess)
    e = launch_apply_cross(ctx->geo, make_ptrs(ctx, frames, out_frames), b, make_cross(x), whole_out != nullptr, st);
  return e == hipSuccess ? RT_OK : hip_fail(e, "cross-channel apply");
}

rt_status rt_frameset_cross(rt_ctx* ctx, const void* const* frames, void* const* out_frames,
                            const rt_stats_buf* stats, const rt_cross_buf* x, void* stream) {
  rt_status r = check_cross_ctx(ctx);
  if (r == RT_OK) r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_frames(ctx, (const void* const*)out_frames, "out_frames");
  if (r == RT_OK) r = check_stats(stats, true, true);
  if (r == RT_OK) r = check_cross(x, true, true, true, true);
  if (r != RT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const Geo& g = ctx->geo;
  const FramePtrs fp = make_ptrs(ctx, frames, out_frames);
  const Bufs b = make_bufs(stats, nullptr, nullptr);
  const CrossBufs xb = make_cross(x);
  hipError_t e = launch_band_stats(g, fp, b, st);
  if (e == hipSuccess) e = launch_cross_stats(g, fp, xb, st);
  if (e == hipSuccess) e = launch_estimate_cross(g, b, xb, st);
  if (e == hipSuccess) e = launch_build_cross(g, xb, st);
  if (e == hipSuccess) e = launch_zero_whole(g, b, st);
  if (e == hipSuccess) e = launch_apply_cross(g, fp, b, xb, true, st);
  return e == hipSuccess ? RT_OK : hip_fail(e, "cross-channel frame-set");
}

rt_status rt_seam_cost(rt_ctx* ctx, const void* const* frames, int32_t factor, double* seam, double* interior,
                       double* rows, int32_t row_stride, void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (factor < 1 || factor > 64) return fail(RT_EINVAL, "factor %d outside 1..64", factor);
  rt_status r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_ptr(seam, 8, "seam");
  if (r == RT_OK) r = check_ptr(interior, 8, "interior");
  if (r != RT_OK) return r;
  int h_max = 0;
  for (const rt_camera_desc& c : ctx->cams) h_max = std::max(h_max, c.height);
  const int max_rows = h_max / factor;
  if (rows) {
    if (!aligned(rows, 8)) return fail(RT_EINVAL, "rows is not 8-byte aligned");
    if (row_stride < max_rows)
      return fail(RT_EINVAL, "row_stride %d < %d rows (max height / factor)", row_stride, max_rows);
  } else {
    // The context's own row buffer, grown when a call needs more rows.
    row_stride = std::max(max_rows, 1);
    const size_t need = (size_t)ctx->n_cams * 2 * row_stride;
    if (need > ctx->seam_rows_n) {
      if (ctx->seam_rows) (void)hipFree(ctx->seam_rows);
      ctx->seam_rows = nullptr;
      ctx->seam_rows_n = 0;
      hipError_t e = hipMalloc((void**)&ctx->seam_rows, need * sizeof(double));
      if (e != hipSuccess) return fail(RT_ENOMEM, "seam cost row buffer: %s", hipGetErrorString(e));
      ctx->seam_rows_n = need;
    }
    rows = ctx->seam_rows;
  }
  const FramePtrs fp = make_ptrs(ctx, frames, nullptr);
  hipError_t e = launch_seam_cost(ctx->geo, fp, seam, interior, rows, row_stride, factor, max_rows,
                                  (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "seam cost");
}

rt_status rt_attention(rt_ctx* ctx, const void* const* frames, const void* const* prev_frames,
                       const rt_attention_opts* ao, uint32_t* cells, uint32_t* windows, uint8_t* selected,
                       void* stream) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (!ao) return fail(RT_EINVAL, "attention options are NULL");
  if (ao->cell < 4 || ao->cell > 256 || ao->cell % 4 != 0)
    return fail(RT_EINVAL, "cell %d must be a multiple of 4 in 4..256", ao->cell);
  if (ao->m < 1 || ao->m > 64) return fail(RT_EINVAL, "m %d outside 1..64", ao->m);
  if (ao->tau < 0 || ao->theta < 0) return fail(RT_EINVAL, "tau and theta must be >= 0");
  rt_status r = check_frames(ctx, frames, "frames");
  if (r == RT_OK) r = check_frames(ctx, prev_frames, "prev_frames");
  if (r == RT_OK) r = check_ptr(cells, 4, "cells");
  if (r != RT_OK) return r;
  if (windows && !aligned(windows, 4)) return fail(RT_EINVAL, "windows is not 4-byte aligned");
  int h_max = 0;
  for (const rt_camera_desc& c : ctx->cams) h_max = std::max(h_max, c.height);
  const int hc = (h_max + ao->cell - 1) / ao->cell, wc = (ctx->w_max + ao->cell - 1) / ao->cell;
  const FramePtrs fp = make_ptrs(ctx, frames, nullptr);
  const FramePtrs pp = make_ptrs(ctx, prev_frames, nullptr);
  hipError_t e = launch_attention(ctx->geo, fp, pp.in, cells, windows, selected, hc, wc, ao->cell, ao->m,
                                  (uint32_t)ao->tau, (uint32_t)ao->theta, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "attention map");
}

rt_status rt_stream_copy(void* dst, const void* src, int64_t bytes, int32_t vec_bytes, void* stream) {
  if (!dst || !src) return fail(RT_EINVAL, "dst or src is NULL");
  if (bytes < 0) return fail(RT_EINVAL, "bytes < 0");
  if (vec_bytes != 4 && vec_bytes != 8 && vec_bytes != 12 && vec_bytes != 16)
    return fail(RT_EINVAL, "vec_bytes must be 4, 8, 12 or 16");
  if (!aligned(dst, 16) || !aligned(src, 16)) return fail(RT_EINVAL, "dst and src must be 16-byte aligned");
  if (bytes >= ((int64_t)1 << 31)) return fail(RT_EUNSUPPORTED, "copies of 2 GiB or more are not supported");
  hipError_t e = launch_stream_copy(dst, src, bytes, vec_bytes, (hipStream_t)stream);
  return e == hipSuccess ? RT_OK : hip_fail(e, "stream copy");
}

rt_status rt_ctx_tuning(const rt_ctx* ctx, int32_t* tile_rows, int32_t* grid, int32_t* n_tiles) {
  if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
  if (tile_rows) *tile_rows = ctx->tile_rows;
  if (grid) *grid = ctx->grid;
  if (n_tiles) *n_tiles = (int32_t)ctx->htiles.size();
  return RT_OK;
}

}  // extern "C"
