/* Driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_oracle_sanitized.py, never part of a product
 * build): every entry point of oracle/rmdf_oracle.c on small configurations,
 * including the degenerate ones (a single pixel, frames smaller than the
 * window, non-finite samples, every velocity mode, odd and even windows).
 * Prints one line per case and "sanitized oracle ok" at the end. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/rmdf_oracle.h"

static unsigned long long rng_state = 0x9e3779b97f4a7c15ull;
static double uniform(void) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(rng_state >> 11) / 9007199254740992.0;
}

static int run_case(int H, int W, int Mx, int My, int Mz, int T, int vmode, int nonfinite) {
  double gx[5] = {-1.0, -0.5, 0.0, 0.5, 1.0}, gy[3] = {-1.0, 0.0, 1.0};
  orc_cfg c;
  c.H = H; c.W = W; c.Mx = Mx; c.My = My; c.Mz = Mz;
  c.Bx = (Mx - 1) / 2 < 2 ? (Mx - 1) / 2 : 2;
  c.By = (My - 1) / 2 < 2 ? (My - 1) / 2 : 2;
  c.dx = Mx / 2; c.dy = My / 2; c.dt = Mz / 2;
  c.alpha = 0.9; c.nvx = 5; c.nvy = 3; c.gx = gx; c.gy = gy;
  c.vmode = vmode; c.fvx = 0.25; c.fvy = -0.5;
  const size_t hw = (size_t)H * W, nv = 15, nb = (size_t)Mx * My * Mz;
  float *fr = malloc(sizeof(float) * hw * T);
  for (size_t i = 0; i < hw * T; ++i) fr[i] = (float)(100.0 + 10.0 * uniform());
  if (nonfinite && hw * T > 3) { fr[1] = NAN; fr[hw * T - 1] = INFINITY; }
  double *out = malloc(sizeof(double) * hw * T), *vxy = malloc(sizeof(double) * hw * T * 2);
  int *idx = malloc(sizeof(int) * hw * T);
  double *rs_last = malloc(sizeof(double) * hw * nv), *r_all = malloc(sizeof(double) * hw * nv * T);
  double *rs_all = malloc(sizeof(double) * hw * nv * T), *en_all = malloc(sizeof(double) * hw * T);
  double complex *spec = malloc(sizeof(double complex) * hw * nb);
  long long nnf = 0;
  const int rc = orc_run(&c, T, fr, out, vxy, idx, rs_last, r_all, rs_all, en_all, spec, &nnf);
  double sum = 0.0;
  for (size_t i = 0; i < hw * T; ++i) sum += fabs(out[i]);
  printf("case %dx%d window %dx%dx%d T=%d vmode=%d: rc=%d nonfinite=%lld sum|out|=%.6g\n", H, W, Mx, My, Mz, T,
         vmode, rc, nnf, sum);
  /* the same configuration with only the required outputs */
  const int rc2 = orc_run(&c, T, fr, out, vxy, idx, NULL, NULL, NULL, NULL, NULL, NULL);
  free(fr); free(out); free(vxy); free(idx); free(rs_last); free(r_all); free(rs_all); free(en_all); free(spec);
  return rc == 0 && rc2 == 0 && (!nonfinite || hw * T <= 3 || nnf == 2) ? 0 : 1;
}

int main(void) {
  int bad = 0;
  bad |= run_case(12, 10, 8, 8, 4, 6, 0, 1);
  bad |= run_case(1, 1, 8, 8, 4, 5, 0, 0);
  bad |= run_case(3, 5, 16, 16, 8, 9, 0, 1);
  bad |= run_case(11, 9, 9, 9, 5, 7, 0, 0);
  bad |= run_case(7, 13, 9, 9, 5, 6, 2, 1);
  bad |= run_case(10, 12, 8, 8, 4, 6, 3, 0);
  bad |= run_case(4, 6, 4, 3, 3, 5, 0, 1);

  /* the single-purpose entry points */
  orc_cfg c = {0};
  double gx[3] = {-1, 0, 1};
  c.H = 4; c.W = 4; c.Mx = 9; c.My = 9; c.Mz = 5; c.Bx = 3; c.By = 3; c.dx = 4; c.dy = 4; c.dt = 2;
  c.alpha = 0.5; c.nvx = 3; c.nvy = 3; c.gx = gx; c.gy = gx;
  double complex *Hk = malloc(sizeof(double complex) * 9 * 9 * 5);
  orc_coeffs(&c, 0.75, -1.25, Hk);
  double complex *S = malloc(sizeof(double complex) * 2 * 9 * 9 * 5);
  for (int i = 0; i < 2 * 9 * 9 * 5; ++i) S[i] = uniform() + I * uniform();
  double R[2 * 9], P[2 * 9 * 9 * 5];
  orc_flow_R(&c, 2, S, R, P);
  orc_flow_R(&c, 2, S, R, NULL);
  double vx = 0, vy = 0;
  orc_refine(&c, R, 4, &vx, &vy);
  orc_refine(&c, R, 0, &vx, &vy);
  orc_refine(&c, R, 8, &vx, &vy);
  double complex s2[12], a0[5], Sobs[12 * 5];
  for (int i = 0; i < 12; ++i) s2[i] = uniform() - 0.5;
  for (int i = 0; i < 5; ++i) a0[i] = 3.0 * uniform();
  orc_observer_series(5, 12, s2, a0, Sobs);
  orc_observer_series(5, 12, s2, NULL, Sobs);
  const double d = orc_dirichlet(5, 0.3) + orc_dirichlet(5, 2.0) + orc_dirichlet(4, 1.0);
  const double v = orc_peak_vertex(-1.0, 1.0, 0.0, 2.0, 1.0, 1.5) + orc_peak_vertex(0, 1, 1, 1, 2, 1);
  printf("entry points: vx=%.6g vy=%.6g dirichlet=%.6g vertex=%.6g\n", vx, vy, d, v);
  free(Hk);
  free(S);
  if (bad) {
    printf("sanitized oracle FAILED\n");
    return 1;
  }
  printf("sanitized oracle ok\n");
  return 0;
}
