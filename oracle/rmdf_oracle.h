/*
 * rmdf_oracle.h - plain FP64 CPU oracle for the recursive multidimensional
 * prediction-error filter (Kennedy, "Parallel software implementation of
 * recursive multidimensional digital filters for point-target detection in
 * cluttered infrared scenes", arXiv:1408.3526).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  It
 * shares no code, header, table or constant with the GPU library and is never
 * linked into it.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg load it.
 *
 * Everything is double precision and written in the order the paper gives:
 *   Sec. 1 and eq. (6)-(7): sliding DFT along rows, then columns (comb +
 *        resonator bank), then a deadbeat observer in time;
 *   Sec. 2, eq. (9)-(10): high-pass, Hann window (frequency-domain
 *        convolution), power spectrum, autocorrelation on the l_z = 1 slice,
 *        first-order smoothing, argmax -> velocity;
 *   Sec. 2, eq. (4), (8): velocity-tuned coefficients at the DFT bins and the
 *        background estimate, eq. (1): output = I(n - m') - Ihat.
 *
 * Window lengths Mx, My, Mz are the DFT sizes per dimension (odd or even).
 */
#ifndef RMDF_ORACLE_H
#define RMDF_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int H, W;            /* frame height (rows, y) and width (columns, x)       */
  int Mx, My, Mz;      /* analysis-window lengths = DFT sizes                 */
  int Bx, By;          /* filter half-bandwidth (Sec. 2, eq. 2); W = 2B+1     */
  int dx, dy, dt;      /* output delay m' (Sec. 3 Parameterization)           */
  double alpha;        /* pole of the first-order smoother of R               */
  int nvx, nvy;        /* candidate-velocity grid sizes                       */
  const double *gx;    /* nvx candidate x-velocities (pixels/frame)           */
  const double *gy;    /* nvy candidate y-velocities                          */
  int vmode;           /* 0: argmax search; 2: fixed velocity (fvx, fvy);
                          3: argmax search, then the peak refined between
                          grid points (orc_refine) and eq. (8) evaluated at
                          the refined, continuous velocity                 */
  double fvx, fvy;
} orc_cfg;

/* Dirichlet kernel of eq. (3), D_W(w) = sin(pi W w) / (W sin(pi w)), with
 * its limit (-1)^((W-1) w) at integer w. */
double orc_dirichlet(int Wn, double w);

/* Eq. (8a)-(8k) evaluated at the DFT bins f = k/M (Sec. 2, the paragraph
 * after eq. 8).  Output Hk[(kx*My + ky)*Mz + kz], kx in [0,Mx) etc.
 * (8h) is read with Delta_z (the printed Delta_x is a typo). */
void orc_coeffs(const orc_cfg *c, double vx, double vy, double complex *Hk);

/* Abscissa of the vertex of the parabola through (x0, r0), (x1, r1), (x2, r2)
 * (x0 < x1 < x2, r1 the largest); x1 when the three values are equal. */
double orc_peak_vertex(double x0, double r0, double x1, double r1, double x2, double r2);

/* Sub-grid velocity (velocity mode 3).  The paper obtains finer velocity
 * resolution by evaluating R at finer, non-integer lags (Sec. 2, the flow
 * paragraph); mode 3 instead interpolates between the grid lags: with the
 * first maximum of the smoothed R at (ix, iy), each axis takes the vertex of
 * the parabola through the peak and its two neighbours along that axis, the
 * other index held fixed.  An axis whose peak is on the grid's edge keeps the
 * grid value.  rsp holds nvy*nvx values, index iy*nvx + ix; grids strictly
 * increasing. */
void orc_refine(const orc_cfg *c, const double *rsp, int best, double *vx, double *vy);

/* Observer of Sec. 1 for one spatial bin over T frames (integrator form).
 * s2[t] is the 2-D spectrum value fed in at frame t; a0 (Mz values, may be
 * NULL = zero) is the initial integrator state a_k(-1).  Writes the observer's
 * spectrum estimate S[t*Mz + kz] = sqrt(Mz) * w^(kz t) a_kz(t). */
void orc_observer_series(int Mz, int T, const double complex *s2,
                         const double complex *a0, double complex *S);

/* Flow part for n local spectra S[i][(kx*My+ky)*Mz+kz] (Sec. 2, eq. 9-10):
 * high-pass, Hann, P = |S'|^2, R on the candidate grid at l_z = 1.
 * R[i][iy*nvx + ix].  Also returns P[i][bin] if P != NULL. */
void orc_flow_R(const orc_cfg *c, int n, const double complex *S, double *R, double *P);

/* Background estimate of eq. (4) for one spectrum and coefficient set. */
double orc_background(const orc_cfg *c, const double complex *Hk,
                      const double complex *S);

/* Whole pipeline over T frames (frames: T*H*W float32, row-major [t][y][x]).
 * Per frame t and anchor (x, y):
 *   out[t][y][x]  = I(t-dt, x-dx, y-dy) - Ihat      (zero outside the frame)
 *   vxy[t][y][x][2] = chosen velocity, idx[t][y][x] = iy*nvx + ix (-1 in vmode 2;
 *                     in vmode 3 the grid peak that was refined)
 * Optional (may be NULL):
 *   rs_last  H*W*nv   smoothed R after the last frame
 *   r_all    T*H*W*nv instantaneous R of every frame
 *   rs_all   T*H*W*nv smoothed R of every frame
 *   en_all   T*H*W    smoothed sum of P (R at zero lag; bounds every |R|)
 *   spec_last H*W*Mx*My*Mz complex spectrum S(k; n) after the last frame
 * Non-finite input samples are replaced by 0 (their count is returned in
 * *n_nonfinite if that pointer is non-NULL).
 * Returns 0 on success, -1 on invalid configuration, -2 on allocation failure. */
int orc_run(const orc_cfg *c, int T, const float *frames,
            double *out, double *vxy, int *idx,
            double *rs_last, double *r_all, double *rs_all, double *en_all,
            double complex *spec_last, long long *n_nonfinite);

/* Number of OpenMP threads the pipeline uses (0 if built without OpenMP). */
int orc_threads(void);
/* Threads for the next parallel regions (n > 0); timing only. */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
