/*
 * ringcorr.h -- C-ABI of the MI355X (gfx950) seam-matched exposure and
 * white-balance correction for a ring of non-overlapping cameras.
 *
 * Method: paper section 3.1 ("White balance and exposure correction").  Narrow
 * bands on both sides of every seam are matched to a shared colour spectrum by
 * one affine map f_c(x) = a_c x + b_c per colour channel, per camera side and
 * per vertical block; each map is blended from the identity at the image
 * centre to f_c at the border over half of the image.  Optional exponential
 * smoothing E = (1 - alpha) E_prev + alpha E_new (alpha = 0.05) of section 3.1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * K        number of cameras of the context (1 .. RT_MAX_CAMS).
 * NB       number of vertical blocks; block j of a camera of height H covers
 *          rows [floor(j H / NB), floor((j + 1) H / NB)).
 * side     0 = left border band (columns [0, B')), 1 = right border band
 *          (columns [W - B', W)), B' = min(band_width, floor(W / 2)).
 * channel  slot c in 0..2; slots >= the camera's channel count are unused
 *          (statistics 0, parameters identity, valid 0).
 * Rings    cameras with equal `ring` form one ring ordered by `pos`
 *          (0 .. m-1, each once): the right side of position p faces the left
 *          side of position p + 1, and in a closed ring the last position
 *          faces position 0.  A one-camera closed ring faces itself.
 *
 * All buffer pointers inside the rt_*_buf structs and all frame pointers are
 * DEVICE pointers owned by the caller; the library never allocates or frees
 * caller-visible memory (a context owns only its own small device tables).
 * Arrays are dense C-order with the shapes given below.  Frames are row-major
 * interleaved: sample (r, col, c) of camera k lives at byte
 *   frame[k] + r * pitch_bytes + (col * channels + c) * bytes_per_sample,
 * bytes_per_sample = 1 for bit_depth 8 and 2 (little-endian uint16) for
 * bit_depth 9..16.  Frame base pointers and pitch_bytes must be multiples of
 * 16; bytes of a row beyond width * channels * bytes_per_sample are neither
 * read nor written.
 *
 * Every compute entry point is asynchronous: it validates its arguments on the
 * host, enqueues kernels on `stream` (a hipStream_t passed as void*, NULL = the
 * default stream) and returns.  Validation failures return a negative status,
 * set rt_last_error() and enqueue nothing.  A HIP launch failure returns
 * RT_EDEVICE.  Nothing aborts and no C++ exception crosses this boundary.  A
 * context is not internally locked: use one context per host thread.  No
 * kernel of the library waits on another workgroup.
 */
#ifndef RINGCORR_H
#define RINGCORR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_MAX_CAMS 64
#define RT_CSLOTS 3
#define RT_NBINS 256
#define RT_MAX_BLOCKS 1024

typedef int32_t rt_status;
enum {
  RT_OK = 0,
  RT_EINVAL = -1,        /* invalid argument: nothing was enqueued */
  RT_ENOMEM = -2,        /* the context could not allocate its device tables */
  RT_EDEVICE = -3,       /* a HIP call failed (launch, copy, graph) */
  RT_EUNSUPPORTED = -4,  /* valid but unsupported combination */
  RT_ESTATE = -5         /* call made on a context in the wrong state */
};

enum { RT_MODE_STANDARD = 0, RT_MODE_SMOOTHING = 1 };

/* Geometry of one camera.  channels is 3 (RGB) or 1; bit_depth 8 (uint8
 * samples) or 9..16 (uint16 samples, channels must be 1).  Every camera of one
 * ring must have the same channels and bit_depth. */
typedef struct {
  int32_t width, height, channels, bit_depth;
  int32_t ring, pos;
  int64_t pitch_bytes;
} rt_camera_desc;

/* Method options.  n_blocks >= 1 (paper: 16 or 64), band_width >= 1 (clamped to
 * floor(W/2) per camera), closed_ring 0/1, mode RT_MODE_*, ema_alpha in (0, 1]
 * (paper: 0.05), 0 < a_min <= a_max (clamp of the gain a).
 * vblend 0/1 (section 5: convex combinations of the maps of adjacent blocks):
 * 1 blends the maps of adjacent blocks row by row in every apply.  With
 * doubled block centres C_j = r0_j + r1_j - 1, row r of block j blends j with
 * its neighbour on r's side of the centre (j - 1 if 2r < C_j, else j + 1;
 * alone before the first centre and from the last one on): between blocks
 * a < b the weight of b is v = round_half_up(256 (2r - C_a) / (C_b - C_a))
 * and each Q16 parameter of the row is floor(((256 - v) P_a + v P_b + 128) /
 * 256) per side and channel; the row's map is then evaluated and blended
 * with the identity as in rt_apply.  Needs height >= n_blocks for every
 * camera (RT_EUNSUPPORTED otherwise).  Estimates and tables are unchanged.
 * fit RT_FIT_* (section 3.1: the affine map makes the main characteristics of
 * the two band distributions agree): RT_FIT_MOMENTS matches the means and
 * standard deviations (see rt_estimate); RT_FIT_QUANTILE fits the line by
 * least squares on M = 64 quantiles: the level-i quantile (i = 0..M-1) of a
 * band histogram h with n samples is the smallest bin v with
 * 2M cum_h(v) >= (2i + 1) n; x_i and f_i are the centres of the own and the
 * facing band's quantile bins in sample units (bin v covers
 * [v 2^s, (v + 1) 2^s) for s = bit_depth - 8, centre v 2^s + (2^s - 1)/2); the
 * shared spectrum's quantiles are y_i = (x_i + f_i)/2 (the midway distribution);
 * a = cov(x, y)/var(x), from exact integer sums and one binary64 division
 * (1 when every x_i is equal), clamped to [a_min, a_max]; b = mean(y) -
 * a mean(x).  Bands that are affine images of each other get the moment
 * fit's map.  The quantile fit is taken by rt_estimate (which then reads
 * stats->band_hist), rt_frameset, rt_frameset_batch, the pipeline and graphs;
 * the object-removal and surrogate entry points return RT_EUNSUPPORTED. */
enum { RT_FIT_MOMENTS = 0, RT_FIT_QUANTILE = 1 };

typedef struct {
  int32_t n_blocks, band_width, closed_ring, mode;
  double ema_alpha, a_min, a_max;
  int32_t vblend, fit;
} rt_opts;

/* Element counts of every caller-owned buffer of a context. */
typedef struct {
  int32_t n_cams, n_blocks, w_max, reserved;
  int64_t band_hist;   /* uint32 [K][2][NB][3][256] */
  int64_t band_sums;   /* uint64 [K][2][NB][3][3] = (n, S1, S2) */
  int64_t whole_hist;  /* uint32 [K][3][256] */
  int64_t whole_sums;  /* uint64 [K][3][3] = (n, S1, S2) */
  int64_t params;      /* double [K][2][NB][3][2] = (a, b) in sample units */
  int64_t valid;       /* uint8  [K][2][NB][3] */
  int64_t lut8;        /* uint8  [K][2][NB][3][256] */
  int64_t q16;         /* int64  [K][2][NB][3][2] = (A, Bq) */
  int64_t weights;     /* uint16 [K][w_max] */
} rt_sizes;

/* Statistics (section 3.1: intensity distributions of the narrow bands along
 * the seams; whole-frame distributions of each camera).  Histogram bin of a
 * sample v: v for 8-bit samples, min(v >> (bit_depth - 8), 255) otherwise.
 * n, S1 = sum v, S2 = sum v^2 are exact. */
typedef struct {
  uint32_t* band_hist;
  uint64_t* band_sums;
  uint32_t* whole_hist;  /* may be NULL where documented */
  uint64_t* whole_sums;  /* may be NULL where documented */
} rt_stats_buf;

/* Per (camera, side, block, channel) affine maps and their history flag
 * (1 = the unit holds an estimate).  This is the device-resident state that
 * exponential smoothing reads and updates. */
typedef struct {
  double* params;
  uint8_t* valid;
} rt_params_buf;

/* Fixed-point maps: q16 (A, Bq) = round_half_even((a, b) * 65536) for every
 * unit; lut8 L[x] = clamp((A x + Bq + 32768) >> 16, 0, 255) for units of 8-bit
 * cameras (entries of 16-bit cameras are not written); weights = Q8 blend
 * weight per column (zero beyond a camera's width). */
typedef struct {
  uint8_t* lut8;
  int64_t* q16;
  uint16_t* weights;
} rt_lut_buf;

typedef struct rt_ctx rt_ctx;

/* Create a context for n_cams cameras.  Validates the rig (dimensions,
 * channels/bit depth, ring positions, pitch) and uploads small device tables
 * to the current HIP device.  *out receives the context; on failure *out is
 * NULL and a negative status is returned. */
rt_status rt_ctx_create(const rt_camera_desc* cams, int32_t n_cams, const rt_opts* opts, rt_ctx** out);

/* Destroy a context (NULL is accepted).  Synchronizes the device first. */
rt_status rt_ctx_destroy(rt_ctx* ctx);

/* Element counts of every buffer this context expects. */
rt_status rt_ctx_sizes(const rt_ctx* ctx, rt_sizes* out);

/* Section 3.1, band statistics: per (camera, side, block, channel) histogram
 * and (n, S1, S2) of the border bands; and, when out->whole_hist and
 * out->whole_sums are both non-NULL, the same over each whole frame.
 * frames: host array of K device pointers.  Outputs are overwritten. */
rt_status rt_stats(rt_ctx* ctx, const void* const* frames, const rt_stats_buf* out, void* stream);

/* Section 3.1, shared spectrum and affine fit, then exponential smoothing.
 * For every (camera, side, block, channel): mu, sigma of the own band and of
 * the facing band (binary64, from n, S1, S2); shared mu_s = (mu_own + mu_fac)/2,
 * sigma_s = (sigma_own + sigma_fac)/2; a = sigma_s/sigma_own (1 if the own
 * variance is 0) clamped to [a_min, a_max]; b = mu_s - a mu_own.  No estimate
 * when either band is empty: the unit keeps its state (identity if invalid).
 * Sides without a facing band (open chain) get the identity.  In smoothing
 * mode a valid unit becomes (1 - alpha) prev + alpha new, element-wise.
 * state is read and overwritten in place (params and valid).  With the
 * context's fit RT_FIT_QUANTILE, (a, b) is the quantile least-squares fit
 * (see rt_opts) of the band histograms stats->band_hist instead. */
rt_status rt_estimate(rt_ctx* ctx, const rt_stats_buf* stats, const rt_params_buf* state, void* stream);

/* Section 3.1, the affine maps as fixed-point tables plus the convex-blend
 * column weights.  weights: h = floor(W/2); column col < h has
 * round_half_up(256 (h - col) / h), col >= W - h has
 * round_half_up(256 (col - W + h + 1) / h), the centre column of an odd width
 * has 0.  All three arrays of `out` are written. */
rt_status rt_build_lut(rt_ctx* ctx, const rt_params_buf* params, const rt_lut_buf* out, void* stream);

/* Section 3.1, the convex blend of the identity and the map over each half
 * image: for every sample x at column col of block j,
 *   y = ((256 - w[col]) x + w[col] f_{side,j,c}(x) + 128) >> 8,
 * with f the 8-bit table (8-bit cameras) or the q16 map clamped to
 * [0, 2^bit_depth - 1] (16-bit cameras); centre columns are copied.
 * out_frames may equal frames (in place).  When whole_out is non-NULL its
 * whole_hist / whole_sums receive the statistics of the INPUT frames, fused
 * into the same pass (its band fields are ignored). */
rt_status rt_apply(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_lut_buf* lut,
                   const rt_stats_buf* whole_out, void* stream);

/* rt_apply with whole-frame statistics for n (1..4) frame-sets in one kernel
 * launch (the launch the fused pipeline issues): frame-set i reads
 * frames[i * K + k] and writes out_frames[i * K + k] for camera k of the
 * context's K cameras, with the tables luts[i]; wholes[i] (whole_hist and
 * whole_sums; band fields ignored) is cleared and receives the statistics of
 * its input.  The same results as n rt_apply calls with whole_out =
 * &wholes[i]; the luts and wholes of different frame-sets must not overlap,
 * and no frame-set may write another's input.  RT_EINVAL for n outside 1..4,
 * RT_EUNSUPPORTED for a context of more than 16 cameras.  For hosts that
 * hold several frame-sets whose tables are built (recorded video). */
rt_status rt_apply_sets(rt_ctx* ctx, int32_t n, const void* const* frames, void* const* out_frames,
                        const rt_lut_buf* luts, const rt_stats_buf* wholes, void* stream);

/* One whole frame-set: band statistics of frame t -> estimate (updating
 * `state`) -> tables and weights, clearing stats' whole-frame fields -> apply
 * to frame t with the whole-frame statistics of the input accumulated in the
 * same pass.  Two kernels, all cameras of all rings batched in each: the
 * first takes each seam block whole (the band statistics of both facing
 * bands, then their estimates and tables), the second applies; no kernel
 * waits on another workgroup.  Same
 * results as rt_stats (bands), rt_estimate, rt_build_lut and rt_apply (with
 * whole statistics) in that order.  stats, state and lut must not overlap
 * each other or the frames. */
rt_status rt_frameset(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_stats_buf* stats,
                      const rt_params_buf* state, const rt_lut_buf* lut, void* stream);

/* rt_frameset over a subset of the cameras, for serving several rigs from one
 * context: bit k of `active` selects camera k (this call only; the
 * context's own set, see rt_ctx_set_active, is not consulted).  Only the
 * active cameras' frames are read (frames[k], out_frames[k] of the others may
 * be NULL), and only their outputs, band and whole statistics, state
 * entries, tables and weights are written; everything of the inactive
 * cameras is left as it was.  A seam's estimate reads both of its bands, so
 * `active` must hold every camera of a ring or none of them (RT_EINVAL
 * otherwise, also for an empty mask or bits at or beyond n_cams).  With all
 * cameras active this is rt_frameset. */
rt_status rt_frameset_batch(rt_ctx* ctx, uint64_t active, const void* const* frames, void* const* out_frames,
                            const rt_stats_buf* stats, const rt_params_buf* state, const rt_lut_buf* lut,
                            void* stream);

/* The frame-set loop with one kernel launch per frame-set (the estimate of
 * frame-set t+1 alongside the apply of frame-set t, as the two-branch graph
 * below, without a graph or a second stream).  In one launch, concurrently:
 *   apply part (frames non-NULL): frames -> out_frames of frame-set t with
 *     the tables in `lut`, built by an earlier call; the statistics of the
 *     input are accumulated into whole's whole_hist / whole_sums, which that
 *     earlier call cleared (band fields ignored);
 *   estimate part (next_frames non-NULL): band statistics of frame-set t+1
 *     into `bands` (band fields; whole fields ignored), the estimate into
 *     `state` (which holds the previous frame-set's estimate for the
 *     temporal smoothing of section 3.1), the
 *     tables and weights into `next_lut`, and next_whole's whole fields
 *     cleared for the call that applies frame-set t+1.
 * At least one part must be requested.  With both, next_lut and next_whole
 * must not share memory with lut and whole (RT_EINVAL when any of their
 * pointers, weights included, are equal), since both parts run at once.  Calls on one stream for
 * t = 0, 1, ..., T with frames = frame-set t-1 (NULL at t = 0) and
 * next_frames = frame-set t (NULL at t = T), alternating two table and two
 * whole-statistics buffers, give exactly the results of T consecutive
 * rt_frameset calls.  Honours the context's active set; the seam and apply
 * parts of the context's configuration (fit, blend) are those of
 * rt_frameset.  All buffers stay owned by the caller. */
rt_status rt_frameset_ahead(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_lut_buf* lut,
                            const rt_stats_buf* whole, const void* const* next_frames, const rt_lut_buf* next_lut,
                            const rt_stats_buf* next_whole, const rt_stats_buf* bands, const rt_params_buf* state,
                            void* stream);

/* Restricts every later call on ctx that takes frames or runs per-camera
 * kernels (all entry points above and below except rt_frameset_batch) to the
 * cameras in `active`, with the semantics rt_frameset_batch documents: the
 * others' frame pointers may be NULL and nothing of theirs is read or
 * written.  Same validity rules as rt_frameset_batch.  After rt_ctx_create
 * every camera is active.  The set is read when a call enqueues its kernels,
 * so work already enqueued (and captured graphs) keep the set they had. */
rt_status rt_ctx_set_active(rt_ctx* ctx, uint64_t active);

/* Frame-set pipeline.  rt_pipe_submit enqueues one frame-set: on the
 * pipeline's own stream E the band statistics, estimate and tables of that
 * frame-set (after `ready_event`, a hipEvent_t passed as void*, if not NULL:
 * the caller records it once the frames are written; stream E does not
 * otherwise wait for the caller's stream), and on the frame-set's lane the
 * apply pass with fused whole-frame statistics, after its tables.  Lanes are
 * taken round-robin: lane 0 is the caller's `stream`, lanes 1.. are streams
 * of the pipeline, so the applies of consecutive frame-sets on different
 * lanes may run concurrently.  Applies are issued `group` frame-sets at a
 * time (when the group is full, or at rt_pipe_join): one cross-stream
 * dependency per lane and group instead of one per frame-set, which is what
 * bounds the host's submission rate; the first `lanes` frame-sets after the
 * pipeline's creation or an rt_pipe_join are issued one at a time, so that
 * an idle pipeline fills at once.  Consecutive frame-sets rotate over
 * `depth` table and whole-frame-statistics slots (luts[depth], wholes[depth],
 * all distinct); the statistics of frame-set t wait for the apply of
 * frame-set t - depth (depth >= 2 * group lets stream E run a group ahead of
 * the applies), so the apply of frame-set t + depth starts only after that of
 * t has finished (frame buffers may be reused from then on).  Band statistics
 * and estimator state are single buffers ordered on stream E, which makes the
 * results exactly those of consecutive rt_frameset calls.  *slot_out (may be
 * NULL) receives the slot of the submitted frame-set; its statistics and
 * tables stay valid until `depth` further submits.  rt_pipe_join(p, stream)
 * issues the pending applies and makes `stream` wait for everything
 * submitted so far; call it before depending on any frame-set's results.
 * 1 <= lanes <= 4, lanes <= depth <= 8, 1 <= group <= depth; rt_pipe_create
 * is lanes = group = 1 (each submit issues its apply on `stream`).  The
 * buffers are caller-owned and must outlive the pipeline; submits of one
 * pipeline must come from one host thread.  A submit on another stream than
 * the previous one first issues the pending applies (lane 0 of those is the
 * stream they were submitted on), so each stream must stay alive until the
 * next submit or rt_pipe_join. */
typedef struct rt_pipe rt_pipe;
rt_status rt_pipe_create(rt_ctx* ctx, int32_t depth, const rt_stats_buf* bands, const rt_params_buf* state,
                         const rt_lut_buf* luts, const rt_stats_buf* wholes, rt_pipe** out);
rt_status rt_pipe_create_lanes(rt_ctx* ctx, int32_t depth, int32_t lanes, int32_t group, const rt_stats_buf* bands,
                               const rt_params_buf* state, const rt_lut_buf* luts, const rt_stats_buf* wholes,
                               rt_pipe** out);
rt_status rt_pipe_submit(rt_pipe* p, const void* const* frames, void* const* out_frames, void* stream,
                         void* ready_event, int32_t* slot_out);
rt_status rt_pipe_join(rt_pipe* p, void* stream);
rt_status rt_pipe_destroy(rt_pipe* p);

/* n consecutive rt_pipe_submit calls (no ready event) in one: frame-set i
 * reads frames[i * K + k] and writes out_frames[i * K + k] for camera k of
 * the context's K cameras.  slots_out (may be NULL) receives the n slots.  A
 * frame-set that fails validation stops the call with its error; the ones
 * before it stay submitted and *n_done (may be NULL) says how many were.
 * For hosts that hold several frame-sets at once (recorded video, a
 * benchmark), it saves one call into the library per frame-set. */
rt_status rt_pipe_submit_n(rt_pipe* p, int32_t n, const void* const* frames, void* const* out_frames, void* stream,
                           int32_t* slots_out, int32_t* n_done);

/* rt_pipe_submit for the cameras in bitmask `active` only (whole rings, as
 * for rt_frameset_batch; the frames and out_frames entries of the other
 * cameras may be NULL), for serving several rigs from one context: the
 * frame-set's statistics, estimate, tables and whole-frame statistics are
 * written for the active cameras and its slot's entries of the others keep
 * their values.  done_event (a hipEvent_t as void*, may be NULL) is recorded
 * on the frame-set's lane right after its apply, so its completion means
 * that this frame-set's outputs and slot are ready; it needs group = 1
 * (RT_EINVAL otherwise). */
rt_status rt_pipe_submit_batch(rt_pipe* p, uint64_t active, const void* const* frames, void* const* out_frames,
                               void* stream, void* ready_event, void* done_event, int32_t* slot_out);

/* Fused applies (fuse = 1; 0, the default, restores the form above): the
 * applies of a group go to one lane, groups taking the lanes in turn, as
 * one kernel launch per run of up to 4 consecutive frame-sets with the same
 * active cameras (the grid holds each frame-set's workgroups in turn, so
 * the launch has no drain between them).  A group then costs the host one
 * cross-stream wait and one record instead of one per lane, and the lanes
 * overlap the end of one group with the start of the next.  Results are
 * those of the unfused pipeline.  Issues the pending applies first.
 * RT_EUNSUPPORTED for a context of more than 16 cameras. */
rt_status rt_pipe_set_fuse(rt_pipe* p, int32_t fuse);

/* ------------------------------------------------------------------------
 * Object removal with the smoothing fallback (section 3.1: the two
 * supplemental methods for objects that move across a seam; section 4.1
 * prefers removal where enough of a block remains, and section 5 leaves the
 * automatic choice between them open - it is made here per seam unit).
 *
 * A band pixel is moving when the absolute difference of one of its samples
 * to the same sample of the previous frame of that camera exceeds
 * tau << (bit_depth - 8) (tau in 8-bit units).  Kept sums: kept_sums uint64
 * [K][2][NB][3][3] = (n, S1, S2) over the band's pixels that do not move
 * (n repeated for every channel of the camera, zero for unused slots).
 * Per seam unit (camera, side, block) the method is
 *   RT_METHOD_REMOVAL   when both facing bands keep at least min_kept of their
 *                       pixels (kept_n / n in binary64): the affine fit of
 *                       rt_estimate from the kept sums, then the context's
 *                       temporal mode;
 *   RT_METHOD_SMOOTHING otherwise: the fit of the whole bands, blended as
 *                       E = (1 - alpha) E_prev + alpha E_new (alpha of the
 *                       context's options; the first estimate taken as is);
 *   RT_METHOD_NONE      without a facing band or with an empty band (the
 *                       state is kept as rt_estimate keeps it).
 * Both sides of a seam take the same method.  method uint8 [K][2][NB].
 * prev_frames NULL: no previous frame-set, nothing moves (kept = whole band).
 * Previous frames have the geometry of the context's cameras.
 * ------------------------------------------------------------------------ */
enum { RT_METHOD_NONE = 0, RT_METHOD_REMOVAL = 1, RT_METHOD_SMOOTHING = 2 };

/* tau >= 0 (paper: a thresholded frame difference; default 20), 0 <= min_kept <= 1
 * (default 0.25). */
typedef struct {
  int32_t tau;
  int32_t reserved;
  double min_kept;
} rt_removal_opts;

/* Band statistics as rt_stats writes them (whole bands; out->whole_* are
 * not used) and the kept sums against prev_frames. */
rt_status rt_motion_stats(rt_ctx* ctx, const void* const* frames, const void* const* prev_frames,
                          const rt_removal_opts* ro, const rt_stats_buf* out, uint64_t* kept_sums, void* stream);

/* The per-unit choice and state update above from stats->band_sums and
 * kept_sums; method may be NULL. */
rt_status rt_estimate_removal(rt_ctx* ctx, const rt_stats_buf* stats, const uint64_t* kept_sums,
                              const rt_removal_opts* ro, const rt_params_buf* state, uint8_t* method, void* stream);

/* rt_frameset with object removal: rt_motion_stats, rt_estimate_removal,
 * rt_build_lut and rt_apply (with whole-frame statistics) in that order, in
 * two kernels as rt_frameset.  Restricted to the context's active set. */
rt_status rt_frameset_removal(rt_ctx* ctx, const void* const* frames, const void* const* prev_frames,
                              void* const* out_frames, const rt_removal_opts* ro, const rt_stats_buf* stats,
                              uint64_t* kept_sums, const rt_params_buf* state, const rt_lut_buf* lut,
                              uint8_t* method, void* stream);

/* Object removal in the frame-set pipeline: with ro (not NULL) every later
 * rt_pipe_submit* estimates as rt_frameset_removal does, each active camera
 * compared with its frame of its last submit (nothing moves in a frame-set
 * in which an active camera has none yet: the first submit after this
 * call, or a camera's first).  kept_sums (uint64 [K][2][NB][3][3]) and
 * method (uint8 [K][2][NB], may be NULL) are single buffers written on the
 * pipeline's stream E in submit order, like the band statistics: after
 * rt_pipe_join they hold the last frame-set's.  The results are exactly
 * those of consecutive rt_frameset_removal calls with prev_frames = the
 * previous frame-set's frames.  A frame-set's input frames are then read
 * again by the next submit's statistics: keep them unchanged until the
 * apply of that next frame-set has finished; an in-place submit (an active
 * camera with out_frames[k] == frames[k]) is refused with RT_EINVAL while
 * removal is on.  ro NULL turns removal off.
 * RT_EUNSUPPORTED unless the context fits the moments. */
rt_status rt_pipe_set_removal(rt_pipe* p, const rt_removal_opts* ro, uint64_t* kept_sums, uint8_t* method);

/* ------------------------------------------------------------------------
 * Cross-channel 3x3 maps (section 5: linear maps across the colour channels
 * instead of one affine map per channel), for contexts whose cameras are all
 * 8-bit RGB (RT_EUNSUPPORTED otherwise, and with vblend or RT_FIT_QUANTILE).
 * Per (camera, side, block) the map is y = M x + t on the pixel's (R, G, B):
 *   the cross sums S_RG, S_RB, S_GB of each band (exact) and its (n, S1, S2)
 *   per channel give the mean mu = S1/n and the covariance C_cd = S_cd/n -
 *   mu_c mu_d (binary64; the diagonal, S2/n - mu^2, clamped at 0); L_own and
 *   L_fac are the lower Cholesky factors of the own and the facing band's C;
 *   the shared spectrum has L* = (L_own + L_fac)/2 and mu* = (mu_own +
 *   mu_fac)/2; M = L* L_own^-1 (solved from M L_own = L*, row by row from the
 *   last column) and t = mu* - M mu_own, so that a band with the own mean and
 *   covariance is sent to one with mean mu* and covariance L* L*^T.  Every
 *   step is one binary64 operation in a fixed order.  When either covariance
 *   has a pivot <= 0, or M has a diagonal entry outside [a_min, a_max] or an
 *   off-diagonal entry beyond a_max in magnitude, M and t are rt_estimate's
 *   per-channel maps (a diagonal M).  An empty band keeps the unit's state
 *   (identity if invalid); a side without a facing band gets the identity.
 *   Smoothing mode blends the twelve parameters as rt_estimate does.
 *   q3 = round_half_even(params3 * 65536); f_r(x) = clamp((A_r0 x_0 + A_r1 x_1
 *   + A_r2 x_2 + B_r + 32768) >> 16, 0, 255); y_r = ((256 - w) x_r + w f_r(x)
 *   + 128) >> 8 with rt_build_lut's column weights.
 * Caller-owned device buffers (element counts): cross uint64 [K][2][NB][3]
 * = (S_RG, S_RB, S_GB); params3 double [K][2][NB][12] = (M row-major, t);
 * valid3 uint8 [K][2][NB]; q3 int64 [K][2][NB][12]; weights uint16
 * [K][w_max].  8-byte alignment (weights 2, valid3 1).
 * ------------------------------------------------------------------------ */
typedef struct {
  uint64_t* cross;
  double* params3;
  uint8_t* valid3;
  int64_t* q3;
  uint16_t* weights;
} rt_cross_buf;

/* Cross sums of every band (x->cross is written). */
rt_status rt_cross_stats(rt_ctx* ctx, const void* const* frames, const rt_cross_buf* x, void* stream);

/* The 3x3 fit from stats->band_sums and x->cross; x->params3 and x->valid3
 * are read and updated in place. */
rt_status rt_estimate_cross(rt_ctx* ctx, const rt_stats_buf* stats, const rt_cross_buf* x, void* stream);

/* x->q3 and x->weights from x->params3. */
rt_status rt_build_cross(rt_ctx* ctx, const rt_cross_buf* x, void* stream);

/* The apply pass with the 3x3 maps of x->q3 and the weights of x->weights;
 * whole_out (may be NULL) receives the whole-frame statistics of the input
 * as in rt_apply. */
rt_status rt_apply_cross(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_cross_buf* x,
                         const rt_stats_buf* whole_out, void* stream);

/* One frame-set with the 3x3 maps: band statistics (stats->band_hist,
 * band_sums), cross sums, fit, maps, then the apply with the whole-frame
 * statistics (stats->whole_hist, whole_sums); the same results as rt_stats,
 * rt_cross_stats, rt_estimate_cross, rt_build_cross and rt_apply_cross in
 * that order. */
rt_status rt_frameset_cross(rt_ctx* ctx, const void* const* frames, void* const* out_frames,
                            const rt_stats_buf* stats, const rt_cross_buf* x, void* stream);

/* ------------------------------------------------------------------------
 * Seam gradient cost (section 4.2, the gradient-cost equation) as a monitor
 * over any frame-set of the context (input or corrected frames).
 *
 * Frames are box-downsampled by `factor` in both directions (8 in the
 * paper; 1..64): each box value is the mean of factor x factor samples.  For
 * a seam between a left image I- and a right image I+, with I-_{-1}, I-_0
 * the last two box columns of I- and I+_0, I+_1 the first two of I+, row i
 * of the downsampled seam has
 *   d+_i = |(I+_1 - I+_0) - (I+_0 - I-_0)|,  d-_i = |(I-_{-1} - I-_0) - (I-_0 - I+_0)|,
 * with |.| the Euclidean norm over the camera's channels in sample units,
 * and the cost is the mean over rows of (d+_i + d-_i) / 2.
 *   seam[k]      the seam between camera k (left image) and the camera its
 *                right side faces (ring order); NaN without one (open
 *                chain end).  A one-camera closed ring faces itself.
 *   interior[k]  the same cost at a virtual seam at column floor(W/2) of
 *                camera k (the reference value of section 4.2's table).
 * The rows of a seam are the boxes of the shorter of its two images from the
 * top; with no row, or an image (or image half) narrower than two boxes, the
 * cost is NaN.  Row values are evaluated in binary64 in the order written
 * above (box means as sum / factor^2, squares summed over the channels in
 * channel order, one square root per norm); the mean sums the rows in a
 * fixed order (deterministic).
 * seam, interior: float64 [K] (8-byte aligned).  rows (may be NULL):
 * float64 [K][2][row_stride], the row values of the seam (index 0) and of
 * the interior (index 1) of each camera; entries past a seam's row count
 * are not written; row_stride >= floor(max height / factor) when rows is
 * given; with rows NULL the context keeps the row values in a device buffer
 * of its own (allocated, or grown, by the first call that needs it).  Only
 * cameras of the active set are read and written.
 * ------------------------------------------------------------------------ */
rt_status rt_seam_cost(rt_ctx* ctx, const void* const* frames, int32_t factor, double* seam, double* interior,
                       double* rows, int32_t row_stride, void* stream);

/* ------------------------------------------------------------------------
 * Difference approach of the attention mechanisms (section 3.3): where to
 * run a detector, from the change between two consecutive frames.
 *
 * A pixel is on when the absolute difference of one of its samples to the
 * same sample of prev_frames exceeds tau << (bit_depth - 8) (tau in 8-bit
 * units, the thresholded difference of section 3.1's object removal).
 * cells u32 [K][hc][wc]: on-pixels per cell of `cell` x `cell` pixels aligned
 * to the frame's top left corner (cut by the border in the last row and
 * column), hc = ceil(max height / cell), wc = ceil(max width / cell) over the
 * context's cameras; entries beyond a camera's own cells are 0.
 * windows u32 and selected u8 [K][hc - m + 1][wc - m + 1] (either may be
 * NULL; both skipped when hc < m or wc < m): the on-pixels of the window of
 * m x m cells starting at each cell, and whether that count exceeds theta;
 * windows that leave a camera's own cell grid are 0 and not selected.
 * cell: a multiple of 4 in 4..256; m in 1..64; tau >= 0; theta >= 0.  Only
 * cameras of the active set are read and written.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t tau, cell, m, theta;
} rt_attention_opts;

rt_status rt_attention(rt_ctx* ctx, const void* const* frames, const void* const* prev_frames,
                       const rt_attention_opts* ao, uint32_t* cells, uint32_t* windows, uint8_t* selected,
                       void* stream);

/* A frame-set captured once into a HIP graph for fixed buffers and replayed
 * with one launch per frame-set.
 *
 * Without next_frames (NULL, next_lut ignored): the graph is rt_frameset on
 * (frames, out_frames) with band statistics in `bands`, estimator state in
 * `state`, tables in `lut` and whole-frame statistics in `whole`.
 *
 * With next_frames: a two-branch graph for software pipelining over
 * consecutive frame-sets t, t+1.  Branch A applies `lut` (estimated by the
 * previous launch) to frame-set t = (frames -> out_frames) with whole-frame
 * statistics into `whole`; branch E, concurrently, computes the band
 * statistics of frame-set t+1 = next_frames into `bands`, the estimate into
 * `state` and the tables into `next_lut` (distinct from `lut`).  Replaying
 * such graphs for t = 0, 1, 2, ... with alternating table buffers, after one
 * rt_stats / rt_estimate / rt_build_lut of frame-set 0, gives exactly the
 * results of consecutive rt_frameset calls.
 *
 * Graph launches of one context must be ordered like its other calls.  A
 * graph becomes invalid (RT_ESTATE at launch) when rt_ctx_tune rebuilds the
 * context's tables; its memory stays owned by the caller and must outlive it. */
typedef struct rt_graph rt_graph;
rt_status rt_graph_create(rt_ctx* ctx, const void* const* frames, void* const* out_frames, const rt_lut_buf* lut,
                          const rt_stats_buf* whole, const void* const* next_frames, const rt_lut_buf* next_lut,
                          const rt_stats_buf* bands, const rt_params_buf* state, rt_graph** out);
rt_status rt_graph_launch(rt_graph* g, void* stream);
rt_status rt_graph_destroy(rt_graph* g);

/* Rebinds the frames of a captured graph for its later launches: frames ->
 * out_frames (validated like rt_frameset's), and for a two-branch graph
 * next_frames (required there, NULL otherwise; RT_EINVAL on a mismatch).
 * Tables, statistics and state buffers stay those of the capture.  One
 * graph then serves any frame buffers: a frame-set costs one rebind (host
 * only: the kernel nodes' frame-pointer arguments are replaced in the
 * instantiated graph) and one launch.  Call it between launches, ordered on
 * the host like them; launches already enqueued keep their frames.
 * RT_EUNSUPPORTED if the capture's frame-pointer arguments could not be
 * identified among the graph's nodes. */
rt_status rt_graph_set_frames(rt_graph* g, const void* const* frames, void* const* out_frames,
                              const void* const* next_frames);

/* Synchronize the device and report RT_EDEVICE if a HIP error is pending. */
rt_status rt_ctx_check(rt_ctx* ctx);

/* Performance knobs that never change results.  grid == 0 (the default):
 * each vertical block of each camera is cut into tiles of equal height of at
 * most tile_rows rows (1..4096), one apply workgroup per tile.  grid > 0
 * (up to 65536): that many workgroups, each on a contiguous share of rows,
 * cut into segments at block boundaries and at most tile_rows rows; with at
 * least one workgroup per camera every camera gets a whole number of shares
 * (one plus its part of the rest by bytes) split evenly by rows, with fewer
 * the shares are equal in bytes and run across cameras.  This balances the
 * work per compute unit when the tile count does not divide evenly over them.
 * Synchronizes the device; rebuilds the context's tables. */
rt_status rt_ctx_tune(rt_ctx* ctx, int32_t tile_rows, int32_t grid);

/* Current knobs (grid as requested, 0 = the default) and the resulting
 * number of apply segments (any pointer may be NULL). */
rt_status rt_ctx_tuning(const rt_ctx* ctx, int32_t* tile_rows, int32_t* grid, int32_t* n_tiles);

/* Instrumentation: with slots > 0, every `every`-th later apply kernel launch
 * of this context (rt_apply, rt_stats with whole-frame statistics,
 * rt_frameset, rt_pipe_submit, fused pipeline applies; the first one
 * included) takes two HIP events
 * attached to its dispatch (the kernel's own start and end, no marker packets
 * around it), kept in a ring of `slots` entries; slots = 0 turns it off.
 * every >= 1.  Synchronizes the device. */
rt_status rt_ctx_timing(rt_ctx* ctx, int32_t slots, int32_t every);

/* Durations in milliseconds of the last min(max_n, recorded, slots) apply
 * kernel launches, oldest first, into ms[]; *n_out receives the count.  Waits
 * for those launches to finish. */
rt_status rt_ctx_apply_times(rt_ctx* ctx, float* ms, int32_t max_n, int32_t* n_out);

/* For the same launches as rt_ctx_apply_times, the number of frame-sets
 * each covered (1, or up to 4 for fused pipeline applies); *n_out receives
 * the count. */
rt_status rt_ctx_apply_sets(const rt_ctx* ctx, int32_t* sets, int32_t max_n, int32_t* n_out);

/* Measurement utility, not part of the method: copy `bytes` bytes from src to
 * dst (device pointers, 16-byte aligned, non-overlapping, bytes < 2 GiB) with
 * vec_bytes (4, 8, 12 or 16) per lane and load/store, the way the apply pass
 * streams frames.  Gives the practical HBM ceiling of a read+write stream of
 * the same size next to the apply pass. */
rt_status rt_stream_copy(void* dst, const void* src, int64_t bytes, int32_t vec_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the estimate (not in the paper; specified here).
 *
 * Unit u3 = (k * 2 + s) * NB + j, a (camera, side, block) of an RGB camera.
 * Input 576 float32 features: regions (0 the whole frame of camera k as
 * passed in - at inference the previous frame-set's, 1 the own band, 2 the
 * facing band of block j, zeros without one) x channels x 64 bins; each bin
 * sums 4 adjacent 256-bins, times 64, divided by the region-channel's sample
 * count, in binary64 rounded once to float32 (a density relative to a flat
 * histogram; zeros for an empty region).
 * Network 576 -> 256 (ReLU) -> 256 (ReLU) -> 6, y = x W + b, row-major
 * weights W[in][out].  Output (a_R, a_G, a_B, b_R/255, b_G/255, b_B/255).
 * Loss: mean of (y - t)^2 over the n x 6 outputs.  The plain estimate judges
 * the network and is its fallback.
 * ------------------------------------------------------------------------ */
#define RT_MLP_IN 576
#define RT_MLP_HID 256
#define RT_MLP_OUT 6

/* Device pointers of one set of network tensors (weights, gradients or Adam moments):
 * w1 [576][256], b1 [256], w2 [256][256], b2 [256], w3 [256][6], b3 [6], float32. */
typedef struct {
  float* w1; float* b1; float* w2; float* b2; float* w3; float* b3;
} rt_mlp;

/* Features of every unit, X float32 [K*2*NB][576] (rows of non-RGB cameras
 * zero), from stats->band_hist (this frame-set) and stats->whole_hist (the
 * whole-frame histograms to use, normally the previous frame-set's); its
 * sums fields are not read and may be NULL. */
rt_status rt_surrogate_features(rt_ctx* ctx, const rt_stats_buf* stats, float* X, void* stream);

/* The plain estimate of section 3.1 before the temporal step: p_new f64
 * [K][2][NB][3][2] (a, b) and status i32 [K][2][NB][3]: 1 new estimate, 0 an
 * empty band (the state is kept), 2 no facing band (identity), 3 unused
 * channel slot.  Reads stats->band_sums only (the other fields may be NULL). */
rt_status rt_estimate_new(rt_ctx* ctx, const rt_stats_buf* stats, double* p_new, int32_t* status, void* stream);

/* Training targets T float32 [K*2*NB][6] from p_new, and mask u8 [K*2*NB]:
 * 1 where the unit is RGB and its three channels hold a new estimate. */
rt_status rt_surrogate_targets(rt_ctx* ctx, const double* p_new, const int32_t* status, float* T, uint8_t* mask,
                               void* stream);

/* Per unit: use the network output Y float32 [K*2*NB][6] iff the unit is
 * eligible (RGB, three new estimates), every output is finite and the
 * residual r = max_c max(|a^ - a|, |b^n - b/255|) against p_new is <= tol
 * (binary64 on the float32 outputs); used units take (a, b) = (a^, 255 b^n).
 * Then the temporal update of `state` exactly as rt_estimate does.  used u8
 * [K*2*NB] and residual f32 [K*2*NB] (inf where not eligible) are written. */
rt_status rt_surrogate_select(rt_ctx* ctx, const float* Y, const double* p_new, const int32_t* status, float tol,
                              const rt_params_buf* state, uint8_t* used, float* residual, void* stream);

/* Device workspace of rt_surrogate_frameset for a context with U = K*2*NB
 * units: X f32 [U][576], H1 and H2 f32 [U][256], Y f32 [U][6], p_new f64
 * [U][3][2], status i32 [U][3], used u8 [U], residual f32 [U].  All owned by
 * the caller; after the call they hold what rt_surrogate_features,
 * rt_estimate_new, rt_mlp_forward and rt_surrogate_select would have written. */
typedef struct {
  float* X; float* H1; float* H2; float* Y;
  double* p_new; int32_t* status; uint8_t* used; float* residual;
} rt_surrogate_work;

/* One frame-set with the learned surrogate in place of the estimate (the
 * data-parallel step of Sec. 3.1 with its per-unit fit predicted): band
 * statistics of `frames` into stats, features against whole_hist_prev
 * (u32 [K][3][256], the previous frame-set's whole-frame histograms; it may
 * be stats->whole_hist itself), plain estimate, network, choice with
 * fallback and temporal update of `state`, tables into `lut`, then the
 * corrected frames and the new whole-frame statistics into stats.  Results
 * are identical to rt_stats (band only), rt_surrogate_features,
 * rt_estimate_new, rt_mlp_forward, rt_surrogate_select, rt_build_lut and
 * rt_apply (with whole-frame statistics) called in turn; six launches
 * instead of eleven.  Restricted to the context's active set (rt_ctx_set_active).
 * Errors: RT_EINVAL for NULL or misaligned pointers or tol < 0 (or NaN). */
rt_status rt_surrogate_frameset(rt_ctx* ctx, const rt_mlp* w, float tol, const void* const* frames,
                                void* const* out_frames, const rt_stats_buf* stats, const uint32_t* whole_hist_prev,
                                const rt_params_buf* state, const rt_lut_buf* lut, const rt_surrogate_work* work,
                                void* stream);

/* rt_surrogate_frameset for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, hosts that forbid
 * allocation after start-up): the same launches and results, with the
 * workspace in a static device array of the library instead of the caller's
 * rt_surrogate_work.  The array holds the workspace of RT_STATIC_UNITS units
 * (K * 2 * NB <= RT_STATIC_UNITS, else RT_EUNSUPPORTED), about 9 MB; each GPU
 * the library runs on holds its own copy until the process ends, set up when
 * the first context on that device is created.  The call allocates nothing.
 * Every call on one GPU shares that GPU's array and its contents of the last
 * call: calls that overlap on one GPU (other streams, other threads) race
 * and must be ordered by the caller.  The context's device must be the
 * current device (RT_EINVAL otherwise). */
#define RT_STATIC_UNITS 2048
rt_status rt_surrogate_frameset_static(rt_ctx* ctx, const rt_mlp* w, float tol, const void* const* frames,
                                       void* const* out_frames, const rt_stats_buf* stats,
                                       const uint32_t* whole_hist_prev, const rt_params_buf* state,
                                       const rt_lut_buf* lut, void* stream);

/* Forward pass over n rows: H1, H2 float32 [n][256] (post-ReLU), Y [n][6]. */
rt_status rt_mlp_forward(const rt_mlp* w, const float* X, int32_t n, float* H1, float* H2, float* Y, void* stream);

/* Gradients of the mean squared error against T [n][6] into `grad`, from the
 * forward pass's X, H1, H2, Y; workspace dY [n][6], dZ1 and dZ2 [n][256]. */
rt_status rt_mlp_backward(const rt_mlp* w, const float* X, const float* H1, const float* H2, const float* Y,
                          const float* T, int32_t n, const rt_mlp* grad, float* dY, float* dZ1, float* dZ2,
                          void* stream);

/* One Adam step (step >= 1 counts steps for the bias correction) updating w, m, v. */
rt_status rt_mlp_adam(const rt_mlp* w, const rt_mlp* grad, const rt_mlp* m, const rt_mlp* v, int32_t step, float lr,
                      float beta1, float beta2, float eps, void* stream);

/* out[0] = mean of (Y - T)^2 over n x 6 values. */
rt_status rt_mlp_mse(const float* Y, const float* T, int32_t n, float* out, void* stream);

/* dst[r] = src[idx[r]] for n rows of row_len floats (mini-batch gather). */
rt_status rt_gather_rows(const float* src, int32_t row_len, const int32_t* idx, int32_t n, float* dst, void* stream);

/* Workspace of rt_mlp_train for mini-batches of `batch` rows, float32 device
 * buffers: xb [batch][576], tb [batch][6], h1, h2, dz1, dz2 [batch][256],
 * y, dy [batch][6]. */
typedef struct {
  float* xb; float* tb; float* h1; float* h2; float* y; float* dy; float* dz1; float* dz2;
} rt_mlp_work;

/* n_steps mini-batch steps of the surrogate's training, enqueued from the
 * library: step s gathers rows idx[s * batch .. (s + 1) * batch) of X
 * [n_rows][576] and T [n_rows][6] (device int32 indices, each < n_rows), runs
 * the forward, the loss (losses[s], device float32), the backward and one Adam
 * step numbered step0 + s (>= 1).  Exactly the sequence of rt_gather_rows,
 * rt_mlp_forward, rt_mlp_backward, rt_mlp_adam and rt_mlp_mse calls per step,
 * without a host round trip between steps. */
rt_status rt_mlp_train(const rt_mlp* w, const rt_mlp* grad, const rt_mlp* m, const rt_mlp* v, const float* X,
                       const float* T, int32_t n_rows, const int32_t* idx, int32_t batch, int32_t n_steps,
                       int32_t step0, float lr, float beta1, float beta2, float eps, const rt_mlp_work* work,
                       float* losses, void* stream);

/* Static description of a status code. */
const char* rt_status_str(rt_status s);

/* Message of the last failure on the calling thread ("" if none). */
const char* rt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RINGCORR_H */
