/* Driver for the library's host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_abi_sanitized.py from a
 * host-only compile of the HIP sources; never part of a product build).  It
 * calls every entry point of include/rmdf.h along its argument-checking
 * paths, which run before any device work, and checks the status each one
 * returns.  Without a GPU a well-formed create reports RMDF_E_DEVICE; with
 * one it succeeds and the context is destroyed again.
 * Prints "sanitized abi ok" when every status is the documented one. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "rmdf.h"

static int failures = 0;

static void expect(const char *what, rmdf_status got, rmdf_status want) {
  if (got != want) {
    printf("MISMATCH %s: got %d, want %d\n", what, (int)got, (int)want);
    ++failures;
  }
}

static rmdf_status create(int H, int W, int Kx, int Ky, int Kt, const float *gx, int nvx, const float *gy, int nvy,
                          const rmdf_params *p) {
  rmdf_ctx *ctx = NULL;
  rmdf_status st = rmdf_create(H, W, Kx, Ky, Kt, gx, nvx, gy, nvy, p, NULL, &ctx);
  if (st == RMDF_OK) rmdf_destroy(ctx);
  if (st != RMDF_OK && rmdf_last_error(NULL)[0] == 0) {
    printf("no message for status %d\n", (int)st);
    ++failures;
  }
  return st;
}

int main(void) {
  const float g[5] = {-1.f, -0.5f, 0.f, 0.5f, 1.f};
  const float gdesc[3] = {1.f, 0.f, -1.f};
  float gbig[40];
  for (int i = 0; i < 40; ++i) gbig[i] = (float)i;
  const float gnan[2] = {0.f, NAN};
  rmdf_params p;
  rmdf_params_default(NULL);
  rmdf_params_default(&p);

  /* rmdf_create: every refusal happens before the device is touched */
  expect("H = 0", create(0, 16, 8, 8, 4, g, 5, g, 5, &p), RMDF_E_INVAL);
  expect("W < 0", create(16, -3, 8, 8, 4, g, 5, g, 5, &p), RMDF_E_INVAL);
  expect("H too large", create(65536, 2, 8, 8, 4, g, 5, g, 5, &p), RMDF_E_INVAL);
  expect("Kx = 1", create(16, 16, 1, 8, 4, g, 5, g, 5, &p), RMDF_E_INVAL);
  expect("NULL grid", create(16, 16, 8, 8, 4, NULL, 5, g, 5, &p), RMDF_E_INVAL);
  expect("empty grid", create(16, 16, 8, 8, 4, g, 0, g, 5, &p), RMDF_E_INVAL);
  expect("grid too long", create(16, 16, 8, 8, 4, gbig, 40, g, 5, &p), RMDF_E_INVAL);
  expect("NaN grid", create(16, 16, 8, 8, 4, gnan, 2, g, 5, &p), RMDF_E_INVAL);
  {
    rmdf_ctx *ctx = NULL;
    expect("out NULL", rmdf_create(16, 16, 8, 8, 4, g, 5, g, 5, &p, NULL, NULL), RMDF_E_INVAL);
    (void)ctx;
  }
  struct { const char *what; rmdf_params q; } bad[16];
  int nb = 0;
  for (int i = 0; i < 16; ++i) rmdf_params_default(&bad[i].q);
  bad[nb].what = "Bx"; bad[nb++].q.Bx = 4;
  bad[nb].what = "By"; bad[nb++].q.By = 9;
  bad[nb].what = "delay_t"; bad[nb++].q.delay_t = 4;
  bad[nb].what = "alpha"; bad[nb++].q.alpha = 1.0f;
  bad[nb].what = "alpha NaN"; bad[nb++].q.alpha = NAN;
  bad[nb].what = "velocity mode"; bad[nb++].q.velocity_mode = 7;
  bad[nb].what = "conf NaN"; bad[nb++].q.conf_threshold = NAN;
  bad[nb].what = "conf > 1"; bad[nb++].q.conf_threshold = 1.5f;
  bad[nb].what = "tile_rows"; bad[nb++].q.tile_rows = -1;
  bad[nb].what = "kernel_variant"; bad[nb++].q.kernel_variant = 5;
  bad[nb].what = "temporal"; bad[nb++].q.temporal = 9;
  bad[nb].what = "fixed velocity"; bad[nb].q.velocity_mode = RMDF_VEL_FIXED; bad[nb++].q.fixed_vx = INFINITY;
  for (int i = 0; i < nb; ++i) expect(bad[i].what, create(16, 16, 8, 8, 4, g, 5, g, 5, &bad[i].q), RMDF_E_INVAL);
  {
    rmdf_params q;
    rmdf_params_default(&q);
    q.velocity_mode = RMDF_VEL_REFINED;
    expect("refined, decreasing grid", create(16, 16, 8, 8, 4, gdesc, 3, g, 5, &q), RMDF_E_INVAL);
    rmdf_params_default(&q);
    q.kernel_variant = 2;
    expect("variant 2 on 8x8x4", create(16, 16, 8, 8, 4, g, 5, g, 5, &q), RMDF_E_UNSUPPORTED);
    rmdf_params_default(&q);
    q.temporal = RMDF_TEMPORAL_RING;
    expect("ring on 8x8x4", create(16, 16, 8, 8, 4, g, 5, g, 5, &q), RMDF_E_UNSUPPORTED);
    rmdf_params_default(&q);
    q.velocity_mode = RMDF_VEL_LEARNED;
    expect("learned on 9x9x5", create(16, 16, 9, 9, 5, g, 5, g, 5, &q), RMDF_E_UNSUPPORTED);
    expect("6x6x3", create(16, 16, 6, 6, 3, g, 5, g, 5, &p), RMDF_E_UNSUPPORTED);
  }
  {
    const rmdf_status st = create(16, 16, 8, 8, 4, g, 5, g, 5, &p);
    if (st != RMDF_OK && st != RMDF_E_DEVICE) expect("well-formed create", st, RMDF_E_DEVICE);
    const rmdf_status s2 = create(16, 16, 8, 8, 4, g, 5, g, 5, NULL);
    if (s2 != RMDF_OK && s2 != RMDF_E_DEVICE) expect("create with defaults", s2, RMDF_E_DEVICE);
  }

  /* calls on a NULL context */
  float *fp = NULL;
  long long n = 0;
  size_t sz = 0;
  double ms = 0;
  int iv = 0;
  expect("push_frame", rmdf_push_frame(NULL, fp), RMDF_E_INVAL);
  expect("push_frames", rmdf_push_frames(NULL, 2, NULL, NULL), RMDF_E_INVAL);
  expect("velocity", rmdf_velocity(NULL, NULL, NULL), RMDF_E_INVAL);
  expect("output", rmdf_output(NULL, NULL), RMDF_E_INVAL);
  expect("frames_pushed", rmdf_frames_pushed(NULL, &n), RMDF_E_INVAL);
  expect("nonfinite_count", rmdf_nonfinite_count(NULL, &n), RMDF_E_INVAL);
  expect("spectrum", rmdf_spectrum(NULL, 1, NULL, NULL, NULL), RMDF_E_INVAL);
  expect("spectrum_noalloc", rmdf_spectrum_noalloc(NULL, 1, NULL, NULL, NULL), RMDF_E_INVAL);
  expect("smoothed_r", rmdf_smoothed_r(NULL, NULL), RMDF_E_INVAL);
  expect("set_timing", rmdf_set_timing(NULL, 1), RMDF_E_INVAL);
  expect("kernel_time", rmdf_kernel_time(NULL, 0, &ms, &n), RMDF_E_INVAL);
  expect("set_weights", rmdf_mlp_set_weights(NULL, NULL, 0), RMDF_E_INVAL);
  expect("features", rmdf_features(NULL, NULL), RMDF_E_INVAL);
  expect("learned_output", rmdf_learned_output(NULL, NULL), RMDF_E_INVAL);
  expect("learned_network", rmdf_learned_network(NULL, NULL, 1, NULL), RMDF_E_INVAL);
  expect("kernel_variant", rmdf_kernel_variant(NULL, &iv), RMDF_E_INVAL);
  expect("tile_rows", rmdf_tile_rows(NULL, &iv), RMDF_E_INVAL);
  expect("coeff_lattice", rmdf_coeff_lattice(NULL, &iv), RMDF_E_INVAL);
  expect("device_bytes", rmdf_device_bytes(NULL, &sz), RMDF_E_INVAL);
  expect("state_bytes", rmdf_state_bytes(NULL, &sz), RMDF_E_INVAL);
  expect("save_state", rmdf_save_state(NULL, NULL, 0), RMDF_E_INVAL);
  expect("load_state", rmdf_load_state(NULL, NULL, 0), RMDF_E_INVAL);
  expect("destroy", rmdf_destroy(NULL), RMDF_OK);
  if (rmdf_last_error(NULL) == NULL) ++failures;

  /* standalone kernels: argument checks */
  unsigned char det[16];
  const float img[16] = {0};
  expect("cfar NULL", rmdf_cfar(NULL, 4, 4, 1, 1, 1.f, det, NULL, NULL), RMDF_E_INVAL);
  expect("cfar size", rmdf_cfar(img, 0, 4, 1, 1, 1.f, det, NULL, NULL), RMDF_E_INVAL);
  expect("cfar window", rmdf_cfar(img, 4, 4, 10, 10, 1.f, det, NULL, NULL), RMDF_E_INVAL);
  expect("cfar k", rmdf_cfar(img, 4, 4, 1, 1, NAN, det, NULL, NULL), RMDF_E_INVAL);
  expect("probe kind", rmdf_hbm_probe(3, img, det, 1024, 4, 0, NULL), RMDF_E_INVAL);
  expect("probe size", rmdf_hbm_probe(2, img, det, 1000, 4, 0, NULL), RMDF_E_INVAL);
  expect("gemm", rmdf_mlp_gemm_nt(NULL, 8, NULL, 8, 1, 1, 8, NULL, 0, NULL, 0, NULL, NULL, 8, NULL), RMDF_E_INVAL);
  expect("transpose", rmdf_mlp_transpose(NULL, NULL, 1, 1, NULL, NULL), RMDF_E_INVAL);
  expect("head", rmdf_mlp_head(NULL, NULL, NULL, NULL, 1, 1.f, 0.5f, NULL, NULL, NULL, NULL, NULL), RMDF_E_INVAL);
  expect("colsum", rmdf_mlp_colsum(NULL, 1, 1, NULL, NULL), RMDF_E_INVAL);
  expect("infer_head", rmdf_mlp_infer_head(NULL, NULL, NULL, 1, NULL, NULL), RMDF_E_INVAL);
  expect("adam", rmdf_mlp_adam(NULL, NULL, NULL, NULL, NULL, 1, 1e-3f, 0.9f, 0.999f, 1e-8f, 1, NULL), RMDF_E_INVAL);
  expect("to_bf16", rmdf_mlp_to_bf16(NULL, NULL, 1, NULL), RMDF_E_INVAL);

  /* batches */
  rmdf_batch *b = NULL;
  rmdf_stream_desc sd[1];
  memset(sd, 0, sizeof sd);
  sd[0].H = 16; sd[0].W = 16; sd[0].Kx = 8; sd[0].Ky = 8; sd[0].Kt = 4;
  sd[0].vgrid_x = g; sd[0].vgrid_y = g; sd[0].nvx = 5; sd[0].nvy = 5;
  expect("batch n = 0", rmdf_batch_create(0, sd, NULL, NULL, &b), RMDF_E_INVAL);
  expect("batch n too large", rmdf_batch_create(5000, sd, NULL, NULL, &b), RMDF_E_INVAL);
  expect("batch NULL descs", rmdf_batch_create(1, NULL, NULL, NULL, &b), RMDF_E_INVAL);
  expect("batch out NULL", rmdf_batch_create(1, sd, NULL, NULL, NULL), RMDF_E_INVAL);
  {
    rmdf_params q;
    rmdf_params_default(&q);
    q.velocity_mode = RMDF_VEL_REFINED;
    const rmdf_status st = rmdf_batch_create(1, sd, &q, NULL, &b);
    if (st != RMDF_E_UNSUPPORTED && st != RMDF_E_DEVICE) expect("batch refined", st, RMDF_E_UNSUPPORTED);
  }
  float *slot = NULL;
  float p50, p99, mean;
  char rep[64];
  rmdf_ctx *sctx = NULL;
  expect("batch_input", rmdf_batch_input(NULL, 0, &slot), RMDF_E_INVAL);
  expect("batch_launch", rmdf_batch_launch(NULL), RMDF_E_INVAL);
  expect("batch_push", rmdf_batch_push(NULL, NULL), RMDF_E_INVAL);
  expect("batch_output", rmdf_batch_output(NULL, 0, NULL, NULL, NULL), RMDF_E_INVAL);
  expect("batch_stream_ctx", rmdf_batch_stream_ctx(NULL, 0, &sctx), RMDF_E_INVAL);
  expect("batch_set_tiles", rmdf_batch_set_tiles(NULL, 0, 8), RMDF_E_INVAL);
  expect("batch_set_schedule", rmdf_batch_set_schedule(NULL, 0), RMDF_E_INVAL);
  expect("batch_autotune", rmdf_batch_autotune(NULL, 1, rep, sizeof rep), RMDF_E_INVAL);
  expect("batch_set_timing", rmdf_batch_set_timing(NULL, 1), RMDF_E_INVAL);
  expect("batch_latency", rmdf_batch_latency(NULL, &p50, &p99, &mean, &n), RMDF_E_INVAL);
  expect("batch_destroy", rmdf_batch_destroy(NULL), RMDF_OK);
  if (rmdf_batch_last_error(NULL) == NULL) ++failures;

  if (failures) {
    printf("sanitized abi FAILED (%d)\n", failures);
    return 1;
  }
  printf("sanitized abi ok\n");
  return 0;
}
