/*
 * rmdf_oracle.c - plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Written for clarity, not speed: every step is the definition or
 * the recursion the paper describes, in the paper's order, on full (not
 * Hermitian-halved) spectra.  Row-parallel OpenMP mirrors the paper's own
 * multicore design (Sec. 5) and changes no arithmetic.
 */
#include "rmdf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846264338327950288;

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 0;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* w_M^k = exp(+j 2 pi k / M), the resonator pole of the sliding DFT (eq. 7). */
static double complex twiddle(int M, long long k) {
  long long r = k % M;
  if (r < 0) r += M;
  return cexp(I * 2.0 * PI * (double)r / (double)M);
}

/* Eq. (3). */
double orc_dirichlet(int Wn, double w) {
  double s = sin(PI * w);
  double r = nearbyint(w);
  if (fabs(w - r) < 1e-12) {
    /* limit at integer w: (-1)^((W-1) w) */
    long long e = ((long long)(Wn - 1)) * (long long)r;
    return (e % 2 == 0) ? 1.0 : -1.0;
  }
  return sin(PI * Wn * w) / (Wn * s);
}

/* Eq. (8a)-(8k) at f = k/M.  Factor tables are built first so that the double
 * sum over the band (8a) is a plain product-sum. */
void orc_coeffs(const orc_cfg *c, double vx, double vy, double complex *Hk) {
  const int Mx = c->Mx, My = c->My, Mz = c->Mz, Bx = c->Bx, By = c->By;
  const int nbx = 2 * Bx + 1, nby = 2 * By + 1;
  const double Dx = 0.5 * (Mx - 1), Dy = 0.5 * (My - 1), Dz = 0.5 * (Mz - 1);
  const double norm = 1.0 / sqrt((double)Mx * My * Mz);

  double complex *bx = malloc(sizeof(double complex) * nbx);
  double complex *by = malloc(sizeof(double complex) * nby);
  double complex *cx = malloc(sizeof(double complex) * Mx);
  double complex *cy = malloc(sizeof(double complex) * My);
  double complex *cz = malloc(sizeof(double complex) * Mz);
  double *dxt = malloc(sizeof(double) * Mx * nbx);
  double *dyt = malloc(sizeof(double) * My * nby);

  for (int j = 0; j < nbx; ++j) { /* (8c) */
    int kp = j - Bx;
    bx[j] = cexp(-I * 2.0 * PI * kp / Mx * (c->dx - Dx));
  }
  for (int j = 0; j < nby; ++j) { /* (8d) */
    int kp = j - By;
    by[j] = cexp(-I * 2.0 * PI * kp / My * (c->dy - Dy));
  }
  for (int k = 0; k < Mx; ++k) cx[k] = cexp(-I * 2.0 * PI * ((double)k / Mx) * Dx); /* (8f) */
  for (int k = 0; k < My; ++k) cy[k] = cexp(-I * 2.0 * PI * ((double)k / My) * Dy); /* (8g) */
  for (int k = 0; k < Mz; ++k) cz[k] = cexp(-I * 2.0 * PI * ((double)k / Mz) * Dz); /* (8h), Delta_z */
  for (int k = 0; k < Mx; ++k) /* (8i) */
    for (int j = 0; j < nbx; ++j)
      dxt[k * nbx + j] = orc_dirichlet(Mx, (double)k / Mx - (double)(j - Bx) / Mx);
  for (int k = 0; k < My; ++k) /* (8j) */
    for (int j = 0; j < nby; ++j)
      dyt[k * nby + j] = orc_dirichlet(My, (double)k / My - (double)(j - By) / My);

  for (int kx = 0; kx < Mx; ++kx)
    for (int ky = 0; ky < My; ++ky)
      for (int kz = 0; kz < Mz; ++kz) {
        double complex acc = 0.0;
        for (int jy = 0; jy < nby; ++jy)
          for (int jx = 0; jx < nbx; ++jx) {
            double phi = vx * (double)(jx - Bx) / Mx + vy * (double)(jy - By) / My;
            double complex bz = cexp(I * 2.0 * PI * phi * (c->dt - Dz));            /* (8e) */
            double dz = orc_dirichlet(Mz, (double)kz / Mz + phi);                 /* (8k) */
            acc += bx[jx] * by[jy] * bz * cx[kx] * cy[ky] * cz[kz] *
                   dxt[kx * nbx + jx] * dyt[ky * nby + jy] * dz;                /* (8b) */
          }
        Hk[(kx * My + ky) * Mz + kz] = norm * acc;                              /* (8a) */
      }
  free(bx); free(by); free(cx); free(cy); free(cz); free(dxt); free(dyt);
}

/* Observer (Sec. 1): integrators in the forward path, feedback of the
 * predicted input, gain 1/Mz so every closed-loop pole sits at z = 0. */
void orc_observer_series(int Mz, int T, const double complex *s2,
                         const double complex *a0, double complex *S) {
  double complex *a = calloc(Mz, sizeof(double complex));
  if (a0) memcpy(a, a0, sizeof(double complex) * Mz);
  const double g = 1.0 / Mz, sq = sqrt((double)Mz);
  for (int t = 0; t < T; ++t) {
    double complex pred = 0.0;
    for (int k = 0; k < Mz; ++k) pred += twiddle(Mz, (long long)k * t) * a[k];
    double complex e = s2[t] - pred;
    for (int k = 0; k < Mz; ++k) a[k] += twiddle(Mz, -(long long)k * t) * e * g;
    for (int k = 0; k < Mz; ++k) S[(size_t)t * Mz + k] = sq * twiddle(Mz, (long long)k * t) * a[k];
  }
  free(a);
}

/* Centred representatives of DFT bin k for the trigonometric evaluation of
 * eq. (10) at non-integer displacement: k itself if |k| < M/2 after
 * centring, or both +M/2 and -M/2 with weight 1/2 for the even-M Nyquist bin. */
static int centred_reps(int M, int k, double *rep, double *wt) {
  if (2 * k == M) { rep[0] = 0.5 * M; rep[1] = -0.5 * M; wt[0] = wt[1] = 0.5; return 2; }
  rep[0] = (2 * k < M) ? k : k - M;
  wt[0] = 1.0;
  return 1;
}

/* cos table for eq. (10) on the l_z = 1 slice: ctab[i*N + bin]. */
static double *build_rtab(const orc_cfg *c) {
  const int Mx = c->Mx, My = c->My, Mz = c->Mz, N = Mx * My * Mz;
  const int nv = c->nvx * c->nvy;
  double *tab = malloc(sizeof(double) * (size_t)nv * N);
  if (!tab) return NULL;
  for (int iy = 0; iy < c->nvy; ++iy)
    for (int ix = 0; ix < c->nvx; ++ix) {
      const double lx = c->gx[ix], ly = c->gy[iy], lz = 1.0;
      double *row = tab + (size_t)(iy * c->nvx + ix) * N;
      for (int kx = 0; kx < Mx; ++kx)
        for (int ky = 0; ky < My; ++ky)
          for (int kz = 0; kz < Mz; ++kz) {
            double rx[2], wx[2], ry[2], wy[2], rz[2], wz[2];
            int nx = centred_reps(Mx, kx, rx, wx);
            int ny = centred_reps(My, ky, ry, wy);
            int nz = centred_reps(Mz, kz, rz, wz);
            double s = 0.0;
            for (int a = 0; a < nx; ++a)
              for (int b = 0; b < ny; ++b)
                for (int d = 0; d < nz; ++d)
                  s += wx[a] * wy[b] * wz[d] *
                       cos(2.0 * PI * (rx[a] * lx / Mx + ry[b] * ly / My + rz[d] * lz / Mz));
            row[(kx * My + ky) * Mz + kz] = s;
          }
    }
  return tab;
}

/* Hann window as a frequency-domain convolution along one axis (Sec. 2):
 * Y(k) = 1/2 X(k) - 1/4 X(k-1) - 1/4 X(k+1), cyclic in k. */
static void hann_axis(const int dims[3], int axis, const double complex *X, double complex *Y) {
  for (int a = 0; a < dims[0]; ++a)
    for (int b = 0; b < dims[1]; ++b)
      for (int d = 0; d < dims[2]; ++d) {
        int idx[3] = {a, b, d};
        int lo[3] = {a, b, d}, hi[3] = {a, b, d};
        lo[axis] = (idx[axis] - 1 + dims[axis]) % dims[axis];
        hi[axis] = (idx[axis] + 1) % dims[axis];
        size_t o = ((size_t)a * dims[1] + b) * dims[2] + d;
        size_t ol = ((size_t)lo[0] * dims[1] + lo[1]) * dims[2] + lo[2];
        size_t oh = ((size_t)hi[0] * dims[1] + hi[1]) * dims[2] + hi[2];
        Y[o] = 0.5 * X[o] - 0.25 * X[ol] - 0.25 * X[oh];
      }
}

static double flow_R_tab(const orc_cfg *c, const double *rtab, const double complex *S,
                         double *R, double *Pout, double complex *w1, double complex *w2) {
  const int Mx = c->Mx, My = c->My, Mz = c->Mz, N = Mx * My * Mz;
  const int dims[3] = {Mx, My, Mz};
  /* high-pass: spatial components with kx = ky = 0 omitted (Sec. 2) */
  memcpy(w1, S, sizeof(double complex) * N);
  for (int kz = 0; kz < Mz; ++kz) w1[kz] = 0.0;
  /* Hann window, one axis at a time (separable) */
  hann_axis(dims, 0, w1, w2);
  hann_axis(dims, 1, w2, w1);
  hann_axis(dims, 2, w1, w2);
  /* eq. (9) */
  double *P = Pout;
  double *Ploc = NULL;
  if (!P) P = Ploc = malloc(sizeof(double) * N);
  double energy = 0.0;
  for (int i = 0; i < N; ++i) {
    P[i] = creal(w2[i]) * creal(w2[i]) + cimag(w2[i]) * cimag(w2[i]);
    energy += P[i];
  }
  /* eq. (10) on the candidate grid, l_z = 1 (real for even P) */
  const int nv = c->nvx * c->nvy;
  for (int i = 0; i < nv; ++i) {
    const double *row = rtab + (size_t)i * N;
    double s = 0.0;
    for (int k = 0; k < N; ++k) s += row[k] * P[k];
    R[i] = s;
  }
  free(Ploc);
  /* sum of P = R at zero lag, an upper bound of |R(l)| for every l */
  return energy;
}

void orc_flow_R(const orc_cfg *c, int n, const double complex *S, double *R, double *P) {
  const int N = c->Mx * c->My * c->Mz, nv = c->nvx * c->nvy;
  double *rtab = build_rtab(c);
#pragma omp parallel
  {
    double complex *w1 = malloc(sizeof(double complex) * N);
    double complex *w2 = malloc(sizeof(double complex) * N);
#pragma omp for
    for (int i = 0; i < n; ++i)
      flow_R_tab(c, rtab, S + (size_t)i * N, R + (size_t)i * nv, P ? P + (size_t)i * N : NULL, w1, w2);
    free(w1); free(w2);
  }
  free(rtab);
}

/* Eq. (4): Ihat = Re sum over kx in [-Bx,Bx], ky in [-By,By], all kz. */
double orc_background(const orc_cfg *c, const double complex *Hk, const double complex *S) {
  const int Mx = c->Mx, My = c->My, Mz = c->Mz;
  double complex acc = 0.0;
  for (int jx = -c->Bx; jx <= c->Bx; ++jx)
    for (int jy = -c->By; jy <= c->By; ++jy)
      for (int kz = 0; kz < Mz; ++kz) {
        int kx = (jx + Mx) % Mx, ky = (jy + My) % My;
        size_t o = ((size_t)kx * My + ky) * Mz + kz;
        acc += Hk[o] * S[o];
      }
  return creal(acc);
}

double orc_peak_vertex(double x0, double r0, double x1, double r1, double x2, double r2) {
  /* r(x) = r1 + b (x - x1) + a (x - x1)^2 through the three points; vertex at
   * x1 - b / (2a).  With h0 = x1 - x0, h2 = x2 - x1:
   *   r0 - r1 = -b h0 + a h0^2,  r2 - r1 = b h2 + a h2^2. */
  const double h0 = x1 - x0, h2 = x2 - x1;
  const double d0 = r0 - r1, d2 = r2 - r1;
  const double a = (d0 * h2 + d2 * h0) / (h0 * h2 * (h0 + h2));
  const double b = (d2 * h0 * h0 - d0 * h2 * h2) / (h0 * h2 * (h0 + h2));
  if (a == 0.0) return x1;
  return x1 - b / (2.0 * a);
}

void orc_refine(const orc_cfg *c, const double *rsp, int best, double *vx, double *vy) {
  const int nvx = c->nvx, nvy = c->nvy, ix = best % nvx, iy = best / nvx;
  *vx = c->gx[ix];
  *vy = c->gy[iy];
  if (ix > 0 && ix < nvx - 1)
    *vx = orc_peak_vertex(c->gx[ix - 1], rsp[best - 1], c->gx[ix], rsp[best], c->gx[ix + 1], rsp[best + 1]);
  if (iy > 0 && iy < nvy - 1)
    *vy = orc_peak_vertex(c->gy[iy - 1], rsp[best - nvx], c->gy[iy], rsp[best], c->gy[iy + 1], rsp[best + nvx]);
}

static int cfg_ok(const orc_cfg *c) {
  if (c->H < 1 || c->W < 1) return 0;
  if (c->Mx < 2 || c->My < 2 || c->Mz < 2) return 0;
  if (c->Mx > 256 || c->My > 256 || c->Mz > 256) return 0;
  if (c->Bx < 0 || c->By < 0 || 2 * c->Bx + 1 > c->Mx || 2 * c->By + 1 > c->My) return 0;
  if (c->dx < 0 || c->dx >= c->Mx || c->dy < 0 || c->dy >= c->My || c->dt < 0 || c->dt >= c->Mz) return 0;
  if (!(c->alpha >= 0.0 && c->alpha < 1.0)) return 0;
  if (c->nvx < 1 || c->nvy < 1 || !c->gx || !c->gy) return 0;
  if (c->vmode != 0 && c->vmode != 2 && c->vmode != 3) return 0;
  if (c->vmode == 3) {
    for (int i = 1; i < c->nvx; ++i) if (!(c->gx[i] > c->gx[i - 1])) return 0;
    for (int i = 1; i < c->nvy; ++i) if (!(c->gy[i] > c->gy[i - 1])) return 0;
  }
  return 1;
}

int orc_run(const orc_cfg *c, int T, const float *frames,
            double *out, double *vxy, int *idx,
            double *rs_last, double *r_all, double *rs_all, double *en_all,
            double complex *spec_last, long long *n_nonfinite) {
  if (!cfg_ok(c) || T < 0 || !frames) return -1;
  const int H = c->H, W = c->W, Mx = c->Mx, My = c->My, Mz = c->Mz;
  const int N = Mx * My * Mz, nv = c->nvx * c->nvy;
  const size_t HW = (size_t)H * W;

  double *img = malloc(sizeof(double) * HW * (size_t)(T > 0 ? T : 1));
  double complex *Sx = malloc(sizeof(double complex) * HW * Mx);
  double complex *S2 = malloc(sizeof(double complex) * HW * Mx * My);
  double complex *a = calloc(HW * (size_t)N, sizeof(double complex));
  double *rs = calloc(HW * (size_t)nv, sizeof(double));
  double *en = calloc(HW, sizeof(double));
  double *rtab = build_rtab(c);
  double complex *Hk = malloc(sizeof(double complex) * (size_t)(nv + 1) * N);
  if (!img || !Sx || !S2 || !a || !rs || !en || !rtab || !Hk) {
    free(img); free(Sx); free(S2); free(a); free(rs); free(en); free(rtab); free(Hk);
    return -2;
  }

  /* coefficient sets: one per candidate, plus the fixed velocity */
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < nv; ++i)
    orc_coeffs(c, c->gx[i % c->nvx], c->gy[i / c->nvx], Hk + (size_t)i * N);
  orc_coeffs(c, c->fvx, c->fvy, Hk + (size_t)nv * N);

  long long bad = 0;
  for (size_t i = 0; i < HW * (size_t)T; ++i) {
    float v = frames[i];
    if (!isfinite(v)) { img[i] = 0.0; ++bad; } else img[i] = (double)v;
  }
  if (n_nonfinite) *n_nonfinite = bad;

  const double sqx = sqrt((double)Mx), sqy = sqrt((double)My), sqz = sqrt((double)Mz);

  for (int t = 0; t < T; ++t) {
    const double *f = img + (size_t)t * HW;

    /* Row sliding DFT (Sec. 1; eq. 6-7): comb x(n) - x(n-M) into a bank of
     * resonators with poles w^k; zero state before the first column. */
#pragma omp parallel for
    for (int y = 0; y < H; ++y) {
      double complex A[256];
      for (int k = 0; k < Mx; ++k) A[k] = 0.0;
      for (int x = 0; x < W; ++x) {
        double comb = f[(size_t)y * W + x] - (x >= Mx ? f[(size_t)y * W + x - Mx] : 0.0);
        for (int k = 0; k < Mx; ++k) {
          A[k] = twiddle(Mx, k) * A[k] + comb;
          Sx[((size_t)y * W + x) * Mx + k] = A[k] / sqx;
        }
      }
    }
    /* Column sliding DFT on the row spectra. */
#pragma omp parallel for
    for (int x = 0; x < W; ++x) {
      double complex B[256];
      for (int kx = 0; kx < Mx; ++kx) {
        for (int k = 0; k < My; ++k) B[k] = 0.0;
        for (int y = 0; y < H; ++y) {
          double complex comb = Sx[((size_t)y * W + x) * Mx + kx] -
                                (y >= My ? Sx[((size_t)(y - My) * W + x) * Mx + kx] : 0.0);
          for (int k = 0; k < My; ++k) {
            B[k] = twiddle(My, k) * B[k] + comb;
            S2[(((size_t)y * W + x) * Mx + kx) * My + k] = B[k] / sqy;
          }
        }
      }
    }

    /* Per pixel: observer, flow, smoothing, argmax, filter (row-parallel). */
#pragma omp parallel
    {
      double complex *S = malloc(sizeof(double complex) * N);
      double complex *w1 = malloc(sizeof(double complex) * N);
      double complex *w2 = malloc(sizeof(double complex) * N);
      double *R = malloc(sizeof(double) * nv);
      double complex *Href = (c->vmode == 3) ? malloc(sizeof(double complex) * N) : NULL;
#pragma omp for
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          const size_t p = (size_t)y * W + x;
          /* temporal deadbeat observer, one per spatial bin (integrator form) */
          for (int kx = 0; kx < Mx; ++kx)
            for (int ky = 0; ky < My; ++ky) {
              double complex *ak = a + p * N + ((size_t)kx * My + ky) * Mz;
              double complex pred = 0.0;
              for (int k = 0; k < Mz; ++k) pred += twiddle(Mz, (long long)k * t) * ak[k];
              double complex e = S2[(p * Mx + kx) * My + ky] - pred;
              for (int k = 0; k < Mz; ++k) ak[k] += twiddle(Mz, -(long long)k * t) * e / (double)Mz;
              for (int k = 0; k < Mz; ++k)
                S[((size_t)kx * My + ky) * Mz + k] = sqz * twiddle(Mz, (long long)k * t) * ak[k];
            }
          if (spec_last && t == T - 1) memcpy(spec_last + p * N, S, sizeof(double complex) * N);

          /* flow: eq. (9)-(10), then the first-order smoother */
          const double e0 = flow_R_tab(c, rtab, S, R, NULL, w1, w2);
          en[p] = (1.0 - c->alpha) * e0 + c->alpha * en[p];
          if (en_all) en_all[(size_t)t * HW + p] = en[p];
          double *rsp = rs + p * nv;
          for (int i = 0; i < nv; ++i) rsp[i] = (1.0 - c->alpha) * R[i] + c->alpha * rsp[i];
          if (r_all) memcpy(r_all + ((size_t)t * HW + p) * nv, R, sizeof(double) * nv);
          if (rs_all) memcpy(rs_all + ((size_t)t * HW + p) * nv, rsp, sizeof(double) * nv);

          /* argmax over the l_z = 1 slice, first maximum wins; v = l / l_z */
          int best = 0;
          for (int i = 1; i < nv; ++i) if (rsp[i] > rsp[best]) best = i;
          double vx, vy;
          const double complex *Hsel;
          if (c->vmode == 2) { vx = c->fvx; vy = c->fvy; Hsel = Hk + (size_t)nv * N; best = -1; }
          else if (c->vmode == 3) {
            orc_refine(c, rsp, best, &vx, &vy);
            orc_coeffs(c, vx, vy, Href);
            Hsel = Href;
          } else { vx = c->gx[best % c->nvx]; vy = c->gy[best / c->nvx]; Hsel = Hk + (size_t)best * N; }
          if (vxy) { vxy[((size_t)t * HW + p) * 2] = vx; vxy[((size_t)t * HW + p) * 2 + 1] = vy; }
          if (idx) idx[(size_t)t * HW + p] = best;

          /* eq. (4) background, eq. (1) prediction error at n - m' */
          double Ihat = orc_background(c, Hsel, S);
          int ts = t - c->dt, xs = x - c->dx, ys = y - c->dy;
          double Id = (ts >= 0 && xs >= 0 && ys >= 0) ? img[(size_t)ts * HW + (size_t)ys * W + xs] : 0.0;
          if (out) out[(size_t)t * HW + p] = Id - Ihat;
        }
      free(S); free(w1); free(w2); free(R); free(Href);
    }
  }
  if (rs_last) memcpy(rs_last, rs, sizeof(double) * HW * nv);
  free(img); free(Sx); free(S2); free(a); free(rs); free(en); free(rtab); free(Hk);
  return 0;
}
