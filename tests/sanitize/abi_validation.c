/* Host-side validation paths of the C-ABI library, run under AddressSanitizer
 * and UndefinedBehaviorSanitizer (the library's host code and this driver are
 * both instrumented; device code is not).  Runs on a machine without a GPU:
 * every call below either fails validation before any HIP call, or reaches
 * the context's device tables and fails there with RT_ENOMEM / RT_EDEVICE
 * after the host-side tables were built.  Exit status 0 when every call
 * returned what it should. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "ringcorr.h"

static int failures = 0;

#define EXPECT(cond, what)                                                 \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "FAILED: %s (last error: %s)\n", what, rt_last_error()); \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static rt_opts default_opts(void) {
  rt_opts o;
  memset(&o, 0, sizeof o);
  o.n_blocks = 16;
  o.band_width = 32;
  o.closed_ring = 1;
  o.mode = RT_MODE_STANDARD;
  o.ema_alpha = 0.05;
  o.a_min = 0.125;
  o.a_max = 8.0;
  return o;
}

static rt_camera_desc cam(int w, int h, int c, int bd, int ring, int pos, int64_t pitch) {
  rt_camera_desc d;
  memset(&d, 0, sizeof d);
  d.width = w;
  d.height = h;
  d.channels = c;
  d.bit_depth = bd;
  d.ring = ring;
  d.pos = pos;
  d.pitch_bytes = pitch;
  return d;
}

/* A creation that must be refused with `want`; the context pointer must be
 * cleared and the message non-empty. */
static void refuse(const rt_camera_desc* cams, int n, const rt_opts* o, rt_status want, const char* what) {
  rt_ctx* ctx = (rt_ctx*)(uintptr_t)0x1234;
  const rt_status st = rt_ctx_create(cams, n, o, &ctx);
  EXPECT(st == want, what);
  EXPECT(ctx == NULL, what);
  EXPECT(strlen(rt_last_error()) > 0, what);
}

/* A valid rig: the host tables are built; without a device the call ends at
 * the device allocation (or succeeds where a device exists). */
static void valid_rig(const rt_camera_desc* cams, int n, const rt_opts* o, const char* what) {
  rt_ctx* ctx = NULL;
  const rt_status st = rt_ctx_create(cams, n, o, &ctx);
  EXPECT(st == RT_OK || st == RT_ENOMEM || st == RT_EDEVICE, what);
  if (st == RT_OK) {
    rt_sizes sz;
    EXPECT(rt_ctx_sizes(ctx, &sz) == RT_OK, what);
    EXPECT(rt_ctx_tune(ctx, 7, 0) == RT_OK, what);
    EXPECT(rt_ctx_tune(ctx, 32, 3 * n + 5) == RT_OK, what);
    EXPECT(rt_ctx_tune(ctx, 16, 1) == RT_OK, what);
    rt_ctx_destroy(ctx);
  } else {
    EXPECT(ctx == NULL, what);
  }
}

int main(void) {
  rt_opts o = default_opts();
  rt_camera_desc good = cam(64, 32, 3, 8, 0, 0, 192);
  rt_camera_desc many[RT_MAX_CAMS + 1];
  for (int i = 0; i <= RT_MAX_CAMS; ++i) many[i] = cam(64, 32, 3, 8, 0, i, 192);

  /* Status strings, including values no status has. */
  EXPECT(strcmp(rt_status_str(RT_OK), "ok") == 0, "status ok");
  EXPECT(strcmp(rt_status_str(-12345), "unknown status") == 0, "unknown status");
  EXPECT(strcmp(rt_status_str(INT32_MIN), "unknown status") == 0, "unknown status min");

  /* Options. */
  refuse(&good, 1, NULL, RT_EINVAL, "NULL options");
  refuse(NULL, 1, &o, RT_EINVAL, "NULL cameras");
  refuse(&good, 0, &o, RT_EINVAL, "no cameras");
  refuse(&good, -7, &o, RT_EINVAL, "negative camera count");
  refuse(many, RT_MAX_CAMS + 1, &o, RT_EINVAL, "too many cameras");
  { rt_opts b = o; b.n_blocks = 0; refuse(&good, 1, &b, RT_EINVAL, "n_blocks 0"); }
  { rt_opts b = o; b.n_blocks = RT_MAX_BLOCKS + 1; refuse(&good, 1, &b, RT_EINVAL, "n_blocks too large"); }
  { rt_opts b = o; b.band_width = -3; refuse(&good, 1, &b, RT_EINVAL, "band_width < 1"); }
  { rt_opts b = o; b.closed_ring = 2; refuse(&good, 1, &b, RT_EINVAL, "closed_ring 2"); }
  { rt_opts b = o; b.mode = 9; refuse(&good, 1, &b, RT_EINVAL, "mode 9"); }
  { rt_opts b = o; b.ema_alpha = 0.0; refuse(&good, 1, &b, RT_EINVAL, "alpha 0"); }
  { rt_opts b = o; b.ema_alpha = 0.0 / 0.0; refuse(&good, 1, &b, RT_EINVAL, "alpha NaN"); }
  { rt_opts b = o; b.a_min = 2.0; b.a_max = 1.0; refuse(&good, 1, &b, RT_EINVAL, "a_min > a_max"); }
  { rt_opts b = o; b.a_max = 1.0 / 0.0; refuse(&good, 1, &b, RT_EINVAL, "a_max inf"); }
  { rt_opts b = o; b.vblend = 2; refuse(&good, 1, &b, RT_EINVAL, "vblend 2"); }
  { rt_opts b = o; b.fit = 7; refuse(&good, 1, &b, RT_EINVAL, "fit 7"); }
  { rt_opts b = o; b.fit = -1; refuse(&good, 1, &b, RT_EINVAL, "fit -1"); }
  {
    rt_camera_desc c = cam(32, 8, 3, 8, 0, 0, 96);
    rt_opts b = o;
    b.vblend = 1;
    refuse(&c, 1, &b, RT_EUNSUPPORTED, "vblend with fewer rows than blocks");
  }

  /* Cameras. */
  { rt_camera_desc c = cam(0, 32, 3, 8, 0, 0, 192); refuse(&c, 1, &o, RT_EINVAL, "width 0"); }
  { rt_camera_desc c = cam(64, -1, 3, 8, 0, 0, 192); refuse(&c, 1, &o, RT_EINVAL, "height -1"); }
  { rt_camera_desc c = cam(40000, 32, 3, 8, 0, 0, 120000); refuse(&c, 1, &o, RT_EINVAL, "width too large"); }
  { rt_camera_desc c = cam(64, 32, 2, 8, 0, 0, 192); refuse(&c, 1, &o, RT_EINVAL, "channels 2"); }
  { rt_camera_desc c = cam(64, 32, 3, 17, 0, 0, 192); refuse(&c, 1, &o, RT_EINVAL, "bit depth 17"); }
  { rt_camera_desc c = cam(64, 32, 3, 12, 0, 0, 400); refuse(&c, 1, &o, RT_EINVAL, "RGB 12-bit"); }
  { rt_camera_desc c = cam(64, 32, 3, 8, 0, 0, 100); refuse(&c, 1, &o, RT_EINVAL, "pitch short"); }
  { rt_camera_desc c = cam(64, 32, 3, 8, 0, 0, 200); refuse(&c, 1, &o, RT_EINVAL, "pitch not 16-aligned"); }
  { rt_camera_desc c = cam(64, 32, 3, 8, 0, 0, -192); refuse(&c, 1, &o, RT_EINVAL, "negative pitch"); }
  { rt_camera_desc c = cam(32768, 32768, 3, 8, 0, 0, 98304); refuse(&c, 1, &o, RT_EUNSUPPORTED, "2 GiB frame"); }
  {
    rt_camera_desc r[2] = {good, good};
    refuse(r, 2, &o, RT_EINVAL, "repeated position");
    r[1].pos = 5;
    refuse(r, 2, &o, RT_EINVAL, "position gap");
    r[1].pos = -1;
    refuse(r, 2, &o, RT_EINVAL, "negative position");
    r[1] = cam(64, 32, 1, 8, 0, 1, 64);
    refuse(r, 2, &o, RT_EINVAL, "ring mixes channels");
  }

  /* NULL arguments of every entry point. */
  EXPECT(rt_ctx_create(&good, 1, &o, NULL) == RT_EINVAL, "NULL out");
  EXPECT(rt_stats(NULL, NULL, NULL, NULL) == RT_EINVAL, "rt_stats NULL");
  EXPECT(rt_estimate(NULL, NULL, NULL, NULL) == RT_EINVAL, "rt_estimate NULL");
  EXPECT(rt_build_lut(NULL, NULL, NULL, NULL) == RT_EINVAL, "rt_build_lut NULL");
  EXPECT(rt_apply(NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "rt_apply NULL");
  EXPECT(rt_frameset(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "rt_frameset NULL");
  EXPECT(rt_frameset_batch(NULL, 1, NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "batch NULL");
  EXPECT(rt_frameset_ahead(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL,
         "ahead NULL");
  EXPECT(rt_ctx_set_active(NULL, 1) == RT_EINVAL, "set_active NULL");
  EXPECT(rt_ctx_sizes(NULL, NULL) == RT_EINVAL, "sizes NULL");
  EXPECT(rt_ctx_destroy(NULL) == RT_OK, "destroy NULL");
  EXPECT(rt_ctx_check(NULL) == RT_EINVAL, "check NULL");
  EXPECT(rt_ctx_tune(NULL, 8, 0) == RT_EINVAL, "tune NULL");
  EXPECT(rt_ctx_tuning(NULL, NULL, NULL, NULL) == RT_EINVAL, "tuning NULL");
  EXPECT(rt_ctx_timing(NULL, 4, 1) == RT_EINVAL, "timing NULL");
  EXPECT(rt_ctx_apply_times(NULL, NULL, 0, NULL) == RT_EINVAL, "apply_times NULL");
  EXPECT(rt_ctx_apply_sets(NULL, NULL, 0, NULL) == RT_EINVAL, "apply_sets NULL");
  EXPECT(rt_pipe_set_fuse(NULL, 1) == RT_EINVAL, "set_fuse NULL");
  EXPECT(rt_pipe_set_removal(NULL, NULL, NULL, NULL) == RT_EINVAL, "set_removal NULL");
  EXPECT(rt_apply_sets(NULL, 1, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "apply_sets NULL");
  EXPECT(rt_graph_set_frames(NULL, NULL, NULL, NULL) == RT_EINVAL, "graph_set_frames NULL");
  EXPECT(rt_stream_copy(NULL, NULL, 16, 16, NULL) == RT_EINVAL, "stream_copy NULL");
  EXPECT(rt_graph_launch(NULL, NULL) == RT_EINVAL, "graph_launch NULL");
  EXPECT(rt_graph_destroy(NULL) == RT_OK, "graph_destroy NULL");
  EXPECT(rt_pipe_submit(NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "pipe_submit NULL");
  EXPECT(rt_pipe_join(NULL, NULL) == RT_EINVAL, "pipe_join NULL");
  EXPECT(rt_pipe_destroy(NULL) == RT_OK, "pipe_destroy NULL");
  EXPECT(rt_motion_stats(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "motion_stats NULL");
  EXPECT(rt_estimate_removal(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "estimate_removal NULL");
  EXPECT(rt_frameset_removal(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL,
         "frameset_removal NULL");
  EXPECT(rt_mlp_forward(NULL, NULL, 1, NULL, NULL, NULL, NULL) == RT_EINVAL, "mlp_forward NULL");
  EXPECT(rt_mlp_mse(NULL, NULL, 1, NULL, NULL) == RT_EINVAL, "mlp_mse NULL");
  EXPECT(rt_gather_rows(NULL, 1, NULL, 1, NULL, NULL) == RT_EINVAL, "gather NULL");
  {
    int32_t done = 5;
    EXPECT(rt_pipe_submit_n(NULL, 2, NULL, NULL, NULL, NULL, &done) == RT_EINVAL && done == 0, "pipe_submit_n NULL");
  }
  EXPECT(rt_cross_stats(NULL, NULL, NULL, NULL) == RT_EINVAL, "cross_stats NULL");
  EXPECT(rt_estimate_cross(NULL, NULL, NULL, NULL) == RT_EINVAL, "estimate_cross NULL");
  EXPECT(rt_build_cross(NULL, NULL, NULL) == RT_EINVAL, "build_cross NULL");
  EXPECT(rt_apply_cross(NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "apply_cross NULL");
  EXPECT(rt_frameset_cross(NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "frameset_cross NULL");
  EXPECT(rt_seam_cost(NULL, NULL, 8, NULL, NULL, NULL, 0, NULL) == RT_EINVAL, "seam_cost NULL");
  EXPECT(rt_attention(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == RT_EINVAL, "attention NULL");

  /* A message longer than the formatting buffer is truncated, not overrun. */
  {
    rt_camera_desc c = cam(64, 32, 3, 8, 123456789, 0, 192);
    rt_camera_desc r[2] = {c, c};
    r[1].pos = 1000000000;
    refuse(r, 2, &o, RT_EINVAL, "large ring and position numbers");
  }

  /* Valid rigs: the host tile tables are built for each (odd sizes, H < NB,
   * the uneven three-ring rig, 64 cameras). */
  valid_rig(&good, 1, &o, "one camera");
  { rt_camera_desc c = cam(1, 1, 3, 8, 0, 0, 16); valid_rig(&c, 1, &o, "1x1"); }
  { rt_camera_desc c = cam(3, 7, 3, 8, 0, 0, 16); rt_opts b = o; b.n_blocks = 64; valid_rig(&c, 1, &b, "H < NB"); }
  {
    rt_camera_desc r[16];
    for (int i = 0; i < 4; ++i) r[i] = cam(4096, 2160, 3, 8, 0, i, 12288);
    for (int i = 0; i < 8; ++i) r[4 + i] = cam(1920, 1080, 3, 8, 1, i, 5760);
    for (int i = 0; i < 4; ++i) r[12 + i] = cam(640, 512, 1, 16, 2, i, 1280);
    valid_rig(r, 16, &o, "uneven rig");
  }
  valid_rig(many, RT_MAX_CAMS, &o, "64 cameras");

  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("abi validation under sanitizers: all checks passed\n");
  return 0;
}
