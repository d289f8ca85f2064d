// rmdf_host.hip - host side of the C ABI declared in include/rmdf.h:
// context lifetime, argument checking, coefficient/twiddle tables (built in
// double precision, rounded to FP32), launch order, optional kernel timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rmdf.h"
#include "rmdf_kernels.h"
#include "rmdf_internal.h"

using cd = std::complex<double>;
static const double kPi = 3.14159265358979323846264338327950288;

namespace {
thread_local std::string g_create_error;

struct EventPair {
  hipEvent_t a, b;
  int which;
};
}  // namespace

struct rmdf_ctx {
  int H = 0, W = 0, MX = 0, MY = 0, MZ = 0, NP = 0, NCOL = 0;
  int nvx = 0, nvy = 0, nv = 0;
  int Bx = 0, By = 0, dx = 0, dy = 0, dt = 0, vmode = 0, TY = 32;
  float alpha = 0.f, fvx = 0.f, fvy = 0.f, conf = 0.9f;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  long long t = 0;
  int nring = 1;
  // device buffers
  float* ring = nullptr;
  float2* rs = nullptr;
  float2* st = nullptr;
  float* rsm = nullptr;
  float* out = nullptr;
  float2* vxy = nullptr;
  int* vidx = nullptr;
  float2 *twx = nullptr, *twy = nullptr, *twz = nullptr, *twA = nullptr;
  float2 *tauy = nullptr, *taux = nullptr, *htab = nullptr;
  float2 *gtab = nullptr, *etab = nullptr;   // lattice factors of htab (16x16x8)
  int* latq = nullptr;
  int lat_q = 0;
  float *gx = nullptr, *gy = nullptr, *tabB = nullptr, *tabC = nullptr;
  int variant = 0;                 // resolved kernel variant (1 generic, 2 wave-per-anchor)
  int write_features = 0;          // plain search that also writes the learned-model input
  int temporal = 0;                // RMDF_TEMPORAL_*: observer state, or ring of 2-D spectra (ring, direct)
  // learned velocity surrogate (16x16x8): features, hidden activations, outputs, weights
  unsigned short* feat = nullptr;  // [HW][1152] BF16
  int* fidx = nullptr;             // [HW] search index (fallback)
  float* vc = nullptr;             // [HW][3] network output (vx, vy, confidence)
  // frame pairs (rmdf_push_frames): the second frame's row spectra, and the
  // first frame's output when the caller gives no buffer for it
  float2* rs2 = nullptr;
  float* out_first = nullptr;
  int* conf_list = nullptr;        // [1 + HW]: count, then the confident anchors (pixel index)
  unsigned short *w1 = nullptr, *w2 = nullptr;   // BF16: W1 in the network kernel's operand order, W2 [64][128]
  float *b1 = nullptr, *b2 = nullptr, *w3 = nullptr, *b3 = nullptr;
  bool weights_set = false;
  bool batch_owned = false;        // advanced by a batch's step, not by pushes
  unsigned long long param_hash = 0;   // grid values and parameters (saved states)
  unsigned long long* nonfinite = nullptr;
  int* xy_scratch = nullptr;
  int xy_cap = 0;
  size_t bytes = 0;
  std::vector<void*> allocs;
  // timing
  int timing = 0;                  // bit w: time kernel w (rmdf_kernel_time numbering)
  std::vector<hipEvent_t> event_pool;   // recycled timing events
  std::vector<EventPair> events;
  double ms[5] = {0, 0, 0, 0, 0};
  long long launches[5] = {0, 0, 0, 0, 0};
  std::string err;
};

static rmdf_status fail(rmdf_ctx* c, rmdf_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return s;
}

static rmdf_status hip_fail(rmdf_ctx* c, hipError_t e, const char* what) {
  return fail(c, RMDF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
static hipError_t dalloc(rmdf_ctx* c, T** p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 1);
  if (e != hipSuccess) return e;
  c->allocs.push_back(q);
  c->bytes += n * sizeof(T);
  *p = static_cast<T*>(q);
  return hipSuccess;
}

static void free_all(rmdf_ctx* c) {
  for (void* p : c->allocs) hipFree(p);
  c->allocs.clear();
  for (auto& ev : c->events) { hipEventDestroy(ev.a); hipEventDestroy(ev.b); }
  c->events.clear();
  for (hipEvent_t e : c->event_pool) hipEventDestroy(e);
  c->event_pool.clear();
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  c->stream = nullptr;
}

// Trigonometric weight of DFT bin k at (possibly non-integer) lag l on M
// points: exp(+j 2 pi kc l / M) for the centred representative kc, and
// cos(pi l) for the even-M Nyquist bin (its two representatives +-M/2 each
// carry half the weight).
static cd trig_weight(int M, int k, double l) {
  if (2 * k == M) return cd(std::cos(kPi * l), 0.0);
  const int kc = (2 * k < M) ? k : k - M;
  const double ph = 2.0 * kPi * kc * l / M;
  return cd(std::cos(ph), std::sin(ph));
}

static double dirichlet(int n, double w) {
  const double r = std::nearbyint(w);
  if (std::fabs(w - r) < 1e-12) {
    const long long e = (long long)(n - 1) * (long long)r;
    return (e % 2 == 0) ? 1.0 : -1.0;
  }
  return std::sin(kPi * n * w) / (n * std::sin(kPi * w));
}

// Background coefficient at bin (kx, ky, kz) for velocity v: the velocity-
// tuned response evaluated at the DFT bins (Sec. 2, eq. 8 with f = k/M).  At
// the bins the spatial Dirichlet factors select the single band term kx'=kx,
// ky'=ky (centred), leaving
//   (MxMyMz)^-1/2 exp(-j2pi(kx m'x/Mx + ky m'y/My)) exp(+j2pi phi (m'z - Dz))
//   exp(-j2pi kz Dz/Mz) D_Mz(kz/Mz + phi),   phi = vx kx/Mx + vy ky/My,
// Dz = (Mz-1)/2.  kx, ky are centred band indices.
static cd coeff(const rmdf_ctx* c, int kx, int ky, int kz, double vx, double vy) {
  const double N = (double)c->MX * c->MY * c->MZ;
  const double phi = vx * kx / c->MX + vy * ky / c->MY;
  const double Dz = 0.5 * (c->MZ - 1);
  const double ph = -2.0 * kPi * ((double)kx * c->dx / c->MX + (double)ky * c->dy / c->MY) +
                    2.0 * kPi * phi * (c->dt - Dz) - 2.0 * kPi * kz * Dz / c->MZ;
  return (dirichlet(c->MZ, (double)kz / c->MZ + phi) / std::sqrt(N)) * cd(std::cos(ph), std::sin(ph));
}

template <class T>
static hipError_t upload(rmdf_ctx* c, T** dst, const std::vector<T>& v) {
  hipError_t e = dalloc(c, dst, v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

static float2 f2(cd z) { return make_float2((float)z.real(), (float)z.imag()); }

static hipError_t build_tables(rmdf_ctx* c, const float* gxh, const float* gyh) {
  hipError_t e;
  std::vector<float2> twx(c->MX), twy(c->MY), twz(c->MZ), twA(c->MZ);
  for (int k = 0; k < c->MX; ++k) twx[k] = f2(std::polar(1.0, 2 * kPi * k / c->MX));
  for (int k = 0; k < c->MY; ++k) twy[k] = f2(std::polar(1.0, 2 * kPi * k / c->MY));
  for (int k = 0; k < c->MZ; ++k) twz[k] = f2(std::polar(1.0, 2 * kPi * k / c->MZ));
  // P = Mz/4096 |h'|^2 (S = sqrt(Mz) X; each axis' Hann is h'/4), l_z = 1
  for (int k = 0; k < c->MZ; ++k) twA[k] = f2(std::polar((double)c->MZ / 4096.0, 2 * kPi * k / c->MZ));
  if ((e = upload(c, &c->twx, twx)) != hipSuccess) return e;
  if ((e = upload(c, &c->twy, twy)) != hipSuccess) return e;
  if ((e = upload(c, &c->twz, twz)) != hipSuccess) return e;
  if ((e = upload(c, &c->twA, twA)) != hipSuccess) return e;

  const int NXH = c->MX / 2 + 1;
  std::vector<float2> tauy((size_t)c->nvy * c->MY), taux((size_t)c->nvx * NXH);
  for (int iy = 0; iy < c->nvy; ++iy)
    for (int k = 0; k < c->MY; ++k) tauy[(size_t)iy * c->MY + k] = f2(trig_weight(c->MY, k, gyh[iy]));
  for (int ix = 0; ix < c->nvx; ++ix)
    for (int k = 0; k < NXH; ++k) {
      // kx and -kx contribute complex-conjugate terms: weight 2 except for
      // the self-conjugate kx = 0 and kx = Mx/2 (even Mx)
      const double w = (k == 0 || 2 * k == c->MX) ? 1.0 : 2.0;
      taux[(size_t)ix * NXH + k] = f2(w * trig_weight(c->MX, k, gxh[ix]));
    }
  if ((e = upload(c, &c->tauy, tauy)) != hipSuccess) return e;
  if ((e = upload(c, &c->taux, taux)) != hipSuccess) return e;

  // background coefficients per candidate (+ the fixed velocity), stored
  // for kx in [0, Bx] (weight 1 for kx = 0, 2 for kx > 0: the -kx terms are
  // conjugates), ky in [-By, By], all kz; sqrt(Mz) folded in (S = sqrt(Mz) X)
  const int nbx = c->Bx + 1, nby = 2 * c->By + 1;
  std::vector<float2> htab((size_t)(c->nv + 1) * nbx * nby * c->MZ);
  const double sz = std::sqrt((double)c->MZ);
  for (int i = 0; i <= c->nv; ++i) {
    const double vx = (i < c->nv) ? gxh[i % c->nvx] : c->fvx;
    const double vy = (i < c->nv) ? gyh[i / c->nvx] : c->fvy;
    for (int kx = 0; kx < nbx; ++kx)
      for (int j = 0; j < nby; ++j)
        for (int kz = 0; kz < c->MZ; ++kz) {
          const double w = (kx == 0) ? 1.0 : 2.0;
          htab[(((size_t)i * nbx + kx) * nby + j) * c->MZ + kz] = f2(w * sz * coeff(c, kx, j - c->By, kz, vx, vy));
        }
  }
  if ((e = upload(c, &c->htab, htab)) != hipSuccess) return e;
  // Lattice factorisation of the same coefficients.  With phi = vx kx/Mx +
  // vy ky/My the coefficient is E(kx, ky) G(phi, kz), E carrying the spatial
  // delay phase and the Hermitian weight, G the temporal part (Dirichlet
  // kernel and phase); G is 1-periodic in phi (the sign of D_Mz(w + 1) and of
  // exp(j 2 pi (m't - Dz)) cancel).  If s*v is an integer for every velocity
  // used (s in {1, 2, 4}), phi = (nx kx + ny ky) / (16 s) mod 1 takes 16 s
  // values, and G becomes a 16s x Mz table.
  if (c->MX == 16 && c->MY == 16 && c->MZ == 8 && c->Bx <= 7 && c->By <= 8) {
    auto on_lattice = [](double v, int s) {
      return std::fabs(v * s) < 16384.0 && std::fabs(v * s - std::nearbyint(v * s)) < 1e-9;
    };
    int s_ok = 0;
    for (int s = 1; s <= 4 && !s_ok; s *= 2) {
      bool ok = true;
      for (int i = 0; i < c->nvx && ok; ++i) ok = on_lattice(gxh[i], s);
      for (int i = 0; i < c->nvy && ok; ++i) ok = on_lattice(gyh[i], s);
      if (c->vmode == 2) ok = ok && on_lattice(c->fvx, s) && on_lattice(c->fvy, s);
      if (ok) s_ok = s;
    }
    if (s_ok) {
      const int Q = 16 * s_ok;
      const double N = 16.0 * 16.0 * 8.0, Dz = 3.5;
      std::vector<float2> gt((size_t)Q * 8), et((size_t)nbx * nby);
      for (int q = 0; q < Q; ++q)
        for (int kz = 0; kz < 8; ++kz) {
          const double phi = (double)q / Q;
          const double ph = 2.0 * kPi * (phi * (c->dt - Dz) - kz * Dz / 8.0);
          gt[(size_t)q * 8 + kz] = f2(sz * dirichlet(8, kz / 8.0 + phi) / std::sqrt(N) * cd(std::cos(ph), std::sin(ph)));
        }
      for (int kx = 0; kx < nbx; ++kx)
        for (int j = 0; j < nby; ++j) {
          const double w = (kx == 0) ? 1.0 : 2.0;
          const double ph = -2.0 * kPi * ((double)kx * c->dx / 16.0 + (double)(j - c->By) * c->dy / 16.0);
          et[(size_t)kx * nby + j] = f2(w * cd(std::cos(ph), std::sin(ph)));
        }
      std::vector<int> lq((size_t)c->nv + 1);
      for (int i = 0; i <= c->nv; ++i) {
        const double vx = (i < c->nv) ? gxh[i % c->nvx] : c->fvx;
        const double vy = (i < c->nv) ? gyh[i / c->nvx] : c->fvy;
        const int nx = (int)std::nearbyint(vx * s_ok), ny = (int)std::nearbyint(vy * s_ok);
        lq[i] = (int)(((unsigned)nx << 16) | ((unsigned)ny & 0xffffu));
      }
      if ((e = upload(c, &c->gtab, gt)) != hipSuccess) return e;
      if ((e = upload(c, &c->etab, et)) != hipSuccess) return e;
      if ((e = upload(c, &c->latq, lq)) != hipSuccess) return e;
      c->lat_q = Q;
    }
  }
  // register-resident weights of the wave-per-anchor 16x16x8 kernel: along
  // ky, cos and sin of 2 pi k l / 16 for k = 1..7 and cos(pi l) (Nyquist);
  // along kx the same with the Hermitian factor 2 folded in
  if (c->MX == 16 && c->MY == 16) {
    std::vector<float> tb((size_t)c->nvy * 16, 0.f), tc((size_t)c->nvx * 16, 0.f);
    for (int iy = 0; iy < c->nvy; ++iy) {
      for (int k = 1; k < 8; ++k) {
        tb[iy * 16 + k - 1] = (float)std::cos(2 * kPi * k * gyh[iy] / 16.0);
        tb[iy * 16 + 6 + k] = (float)std::sin(2 * kPi * k * gyh[iy] / 16.0);
      }
      tb[iy * 16 + 14] = (float)std::cos(kPi * gyh[iy]);
    }
    for (int ix = 0; ix < c->nvx; ++ix) {
      for (int k = 1; k < 8; ++k) {
        tc[ix * 16 + k - 1] = (float)(2.0 * std::cos(2 * kPi * k * gxh[ix] / 16.0));
        tc[ix * 16 + 6 + k] = (float)(2.0 * std::sin(2 * kPi * k * gxh[ix] / 16.0));
      }
      tc[ix * 16 + 14] = (float)std::cos(kPi * gxh[ix]);
    }
    if ((e = upload(c, &c->tabB, tb)) != hipSuccess) return e;
    if ((e = upload(c, &c->tabC, tc)) != hipSuccess) return e;
  }
  std::vector<float> gx(gxh, gxh + c->nvx), gy(gyh, gyh + c->nvy);
  if ((e = upload(c, &c->gx, gx)) != hipSuccess) return e;
  if ((e = upload(c, &c->gy, gy)) != hipSuccess) return e;
  return hipSuccess;
}

rmdf::PixArgs rmdf_internal_pixargs(const rmdf_ctx* c) {
  rmdf::PixArgs a{};
  a.H = c->H; a.W = c->W; a.TY = c->TY;
  a.nvx = c->nvx; a.nvy = c->nvy; a.nv = c->nv;
  a.bx = c->Bx; a.by = c->By; a.dx = c->dx; a.dy = c->dy;
  a.vmode = c->vmode;
  a.alpha = c->alpha; a.inv_sqrt_my = (float)(1.0 / std::sqrt((double)c->MY));
  a.fvx = c->fvx; a.fvy = c->fvy;
  a.rs = c->rs; a.st = c->st; a.rsm = c->rsm;
  a.ring_delayed = nullptr;
  a.out = c->out; a.vxy = c->vxy; a.vidx = c->vidx;
  a.twy = c->twy; a.twz = c->twz; a.twA = c->twA; a.tauy = c->tauy; a.taux = c->taux; a.htab = c->htab;
  a.gx = c->gx; a.gy = c->gy; a.tabB = c->tabB; a.tabC = c->tabC;
  a.feat = c->feat; a.fidx = c->fidx; a.dt = c->dt;
  a.gtab = c->gtab; a.etab = c->etab; a.latq = c->latq; a.lat_q = c->lat_q;
  return a;
}
const float* rmdf_internal_ring(const rmdf_ctx* c, int* nring, int* dt) {
  *nring = c->nring;
  *dt = c->dt;
  return c->ring;
}
const float2* rmdf_internal_twx(const rmdf_ctx* c) { return c->twx; }
unsigned long long* rmdf_internal_nonfinite(const rmdf_ctx* c) { return c->nonfinite; }
void rmdf_internal_shape(const rmdf_ctx* c, int* mx, int* my, int* mz, int* variant) {
  *mx = c->MX; *my = c->MY; *mz = c->MZ; *variant = c->variant;
}
void rmdf_internal_advance(rmdf_ctx* c) { c->t += 1; }
void rmdf_internal_set_batch_owned(rmdf_ctx* c) { c->batch_owned = true; }

// FNV-1a over raw bytes (identifies the configuration a saved state belongs to).
static unsigned long long fnv1a(unsigned long long h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

// Frame pairs run on the 16x16x8 one-wavefront-per-anchor kernel in its
// observer form with the search or a fixed velocity.
static bool pairs_supported(const rmdf_ctx* c) {
  return c->variant == 2 && c->temporal == RMDF_TEMPORAL_OBSERVER &&
         (c->vmode == RMDF_VEL_SEARCH || c->vmode == RMDF_VEL_FIXED) && !c->write_features;
}
void rmdf_internal_set_create_error(const std::string& m) { g_create_error = m; }

extern "C" {

void rmdf_params_default(rmdf_params* p) {
  if (!p) return;
  p->Bx = p->By = -1;
  p->delay_x = p->delay_y = p->delay_t = -1;
  p->alpha = -1.0f;
  p->velocity_mode = RMDF_VEL_SEARCH;
  p->fixed_vx = p->fixed_vy = 0.0f;
  p->conf_threshold = 0.9f;
  p->tile_rows = 0;
  p->kernel_variant = 0;
  p->write_features = 0;
  p->temporal = RMDF_TEMPORAL_OBSERVER;
}

rmdf_status rmdf_create(int H, int W, int Kx, int Ky, int Kt, const float* vgrid_x, int nvx, const float* vgrid_y,
                        int nvy, const rmdf_params* pin, void* hip_stream, rmdf_ctx** out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, RMDF_E_INVAL, "out is NULL");
  *out = nullptr;
  if (H < 1 || W < 1) return fail(nullptr, RMDF_E_INVAL, "frame size must be at least 1x1");
  if (H > 65535) return fail(nullptr, RMDF_E_INVAL, "frame height must be <= 65535");
  if (Kx < 2 || Ky < 2 || Kt < 2) return fail(nullptr, RMDF_E_INVAL, "window lengths must be >= 2");
  if (!vgrid_x || !vgrid_y) return fail(nullptr, RMDF_E_INVAL, "velocity grid pointer is NULL");
  if (nvx < 1 || nvy < 1 || nvx > rmdf::NVX_MAX || nvy > rmdf::NVY_MAX)
    return fail(nullptr, RMDF_E_INVAL, "velocity grid sizes must be in [1, 33]");
  for (int i = 0; i < nvx; ++i)
    if (!std::isfinite(vgrid_x[i])) return fail(nullptr, RMDF_E_INVAL, "non-finite velocity grid value");
  for (int i = 0; i < nvy; ++i)
    if (!std::isfinite(vgrid_y[i])) return fail(nullptr, RMDF_E_INVAL, "non-finite velocity grid value");
  rmdf_params p;
  if (pin) p = *pin;
  else rmdf_params_default(&p);
  const int Bx = p.Bx < 0 ? (3 * Kx) / 8 : p.Bx;
  const int By = p.By < 0 ? (3 * Ky) / 8 : p.By;
  if (Bx > (Kx - 1) / 2 || By > (Ky - 1) / 2) return fail(nullptr, RMDF_E_INVAL, "B must be <= floor((M-1)/2)");
  const int dx = p.delay_x < 0 ? Kx / 2 : p.delay_x;
  const int dy = p.delay_y < 0 ? Ky / 2 : p.delay_y;
  const int dt = p.delay_t < 0 ? Kt / 2 : p.delay_t;
  if (dx >= Kx || dy >= Ky || dt >= Kt) return fail(nullptr, RMDF_E_INVAL, "delay m' must be < M");
  const float alpha = p.alpha < 0.f ? std::exp(-0.1f) : p.alpha;
  if (!(alpha >= 0.f && alpha < 1.f)) return fail(nullptr, RMDF_E_INVAL, "alpha must be in [0, 1)");
  if (p.velocity_mode < RMDF_VEL_SEARCH || p.velocity_mode > RMDF_VEL_REFINED)
    return fail(nullptr, RMDF_E_INVAL, "unknown velocity mode");
  if (p.velocity_mode == RMDF_VEL_REFINED) {
    for (int i = 1; i < nvx; ++i)
      if (!(vgrid_x[i] > vgrid_x[i - 1])) return fail(nullptr, RMDF_E_INVAL, "refined velocity needs strictly increasing grids");
    for (int i = 1; i < nvy; ++i)
      if (!(vgrid_y[i] > vgrid_y[i - 1])) return fail(nullptr, RMDF_E_INVAL, "refined velocity needs strictly increasing grids");
    if (p.write_features)
      return fail(nullptr, RMDF_E_UNSUPPORTED, "write_features needs velocity mode 0");
  }
  if (!(p.conf_threshold >= 0.f && p.conf_threshold <= 1.f))
    return fail(nullptr, RMDF_E_INVAL, "conf_threshold must be a finite value in [0, 1]");
  if (p.velocity_mode == RMDF_VEL_FIXED && !(std::isfinite(p.fixed_vx) && std::isfinite(p.fixed_vy)))
    return fail(nullptr, RMDF_E_INVAL, "fixed velocity must be finite");
  if (p.tile_rows < 0) return fail(nullptr, RMDF_E_INVAL, "tile_rows must be >= 0");
  if (p.kernel_variant < 0 || p.kernel_variant > 2) return fail(nullptr, RMDF_E_INVAL, "kernel_variant must be 0, 1 or 2");
  const bool w16 = rmdf::pixel16_eligible(Kx, Ky, Kt, nvx, nvy);
  if (p.kernel_variant == 2 && !w16)
    return fail(nullptr, RMDF_E_UNSUPPORTED, "kernel_variant 2 needs a 16x16x8 window and at most 21 candidates per axis");
  if (p.temporal != RMDF_TEMPORAL_OBSERVER && p.temporal != RMDF_TEMPORAL_RING && p.temporal != RMDF_TEMPORAL_DIRECT)
    return fail(nullptr, RMDF_E_INVAL, "unknown temporal mode");
  if (p.temporal != RMDF_TEMPORAL_OBSERVER) {
    if (!w16 || p.kernel_variant == 1)
      return fail(nullptr, RMDF_E_UNSUPPORTED,
                  "the temporal ring and the direct spectrum need the 16x16x8 window, kernel variant 2 and at most 21 "
                  "candidates per axis");
    if ((p.velocity_mode != RMDF_VEL_SEARCH && p.velocity_mode != RMDF_VEL_FIXED) || p.write_features)
      return fail(nullptr, RMDF_E_UNSUPPORTED,
                  "the temporal ring and the direct spectrum support the search and fixed velocity modes");
  }
  const bool needs16 = (p.velocity_mode == RMDF_VEL_LEARNED) || p.write_features;
  if (needs16 && (!w16 || p.kernel_variant == 1))
    return fail(nullptr, RMDF_E_UNSUPPORTED,
                "the learned velocity model and its features need the 16x16x8 window, kernel variant 2 and at most 21 candidates per axis");
  if (!rmdf::shape_supported(Kx, Ky, Kt))
    return fail(nullptr, RMDF_E_UNSUPPORTED, "window shape has no compiled kernel (8x8x4, 16x16x8, 9x9x5)");

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) return fail(nullptr, RMDF_E_DEVICE, "no HIP device available");

  rmdf_ctx* c = new (std::nothrow) rmdf_ctx();
  if (!c) return fail(nullptr, RMDF_E_NOMEM, "host allocation failed");
  hipGetDevice(&c->device);
  c->H = H; c->W = W; c->MX = Kx; c->MY = Ky; c->MZ = Kt;
  c->NP = rmdf::planes_for(Kx);
  c->NCOL = c->NP * Ky;
  c->nvx = nvx; c->nvy = nvy; c->nv = nvx * nvy;
  c->Bx = Bx; c->By = By; c->dx = dx; c->dy = dy; c->dt = dt;
  c->alpha = alpha; c->vmode = p.velocity_mode; c->fvx = p.fixed_vx; c->fvy = p.fixed_vy;
  c->conf = p.conf_threshold;
  c->variant = p.kernel_variant != 0 ? p.kernel_variant : (w16 ? 2 : 1);
  c->TY = p.tile_rows > 0 ? p.tile_rows
                          : rmdf::auto_tile_rows(H, W, c->variant == 2 ? rmdf::p16_block_columns()
                                                                        : rmdf::pixel_block_columns(Kx, Ky, Kt));
  c->write_features = p.write_features ? 1 : 0;
  c->temporal = p.temporal;
  {
    unsigned long long h = 0xcbf29ce484222325ull;
    h = fnv1a(h, vgrid_x, sizeof(float) * nvx);
    h = fnv1a(h, vgrid_y, sizeof(float) * nvy);
    const int iv[8] = {Bx, By, dx, dy, dt, p.velocity_mode, c->write_features, c->variant};
    const float fv[3] = {alpha, p.fixed_vx, p.fixed_vy};
    h = fnv1a(h, iv, sizeof iv);
    c->param_hash = fnv1a(h, fv, sizeof fv);
  }
  // one slot beyond the delay: a frame pair stores its second frame before
  // the pair's first frame has read its delayed sample
  c->nring = dt + 2;
  // NULL: the device's default (null) stream, which is also torch's default
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->own_stream = false;
  const size_t HW = (size_t)H * W;
  auto bail = [&](hipError_t err, const char* what) {
    rmdf_status s = (err == hipErrorOutOfMemory || err == hipErrorMemoryAllocation)
                        ? fail(nullptr, RMDF_E_NOMEM, std::string(what) + ": out of device memory")
                        : hip_fail(nullptr, err, what);
    free_all(c);
    delete c;
    return s;
  };
  if ((e = dalloc(c, &c->ring, HW * c->nring)) != hipSuccess) return bail(e, "ring");
  if ((e = dalloc(c, &c->rs, HW * c->NP)) != hipSuccess) return bail(e, "row spectra");
  if ((e = dalloc(c, &c->st, HW * c->NCOL * Kt)) != hipSuccess) return bail(e, "observer state");
  if ((e = dalloc(c, &c->rsm, HW * c->nv)) != hipSuccess) return bail(e, "smoothed autocorrelation");
  if ((e = dalloc(c, &c->out, HW)) != hipSuccess) return bail(e, "output");
  if ((e = dalloc(c, &c->vxy, HW)) != hipSuccess) return bail(e, "velocity");
  if ((e = dalloc(c, &c->vidx, HW)) != hipSuccess) return bail(e, "velocity index");
  if ((e = dalloc(c, &c->nonfinite, 1)) != hipSuccess) return bail(e, "counter");
  if ((e = build_tables(c, vgrid_x, vgrid_y)) != hipSuccess) return bail(e, "tables");
  if (needs16 && (e = dalloc(c, &c->feat, HW * 1152)) != hipSuccess) return bail(e, "features");
  if (pairs_supported(c)) {
    if ((e = dalloc(c, &c->rs2, HW * c->NP)) != hipSuccess) return bail(e, "row spectra");
    if ((e = dalloc(c, &c->out_first, HW)) != hipSuccess) return bail(e, "output");
  }
  if (c->vmode == RMDF_VEL_LEARNED) {
    if ((e = dalloc(c, &c->fidx, HW)) != hipSuccess) return bail(e, "fallback index");
    if ((e = dalloc(c, &c->vc, HW * 3)) != hipSuccess) return bail(e, "network output");
    if ((e = dalloc(c, &c->conf_list, HW + 1)) != hipSuccess) return bail(e, "confident-anchor list");
    if ((e = dalloc(c, &c->w1, (size_t)128 * 1152)) != hipSuccess) return bail(e, "weights");
    if ((e = dalloc(c, &c->w2, (size_t)64 * 128)) != hipSuccess) return bail(e, "weights");
    if ((e = dalloc(c, &c->b1, 128)) != hipSuccess) return bail(e, "weights");
    if ((e = dalloc(c, &c->b2, 64)) != hipSuccess) return bail(e, "weights");
    if ((e = dalloc(c, &c->w3, 192)) != hipSuccess) return bail(e, "weights");
    if ((e = dalloc(c, &c->b3, 3)) != hipSuccess) return bail(e, "weights");
  }
  // zero the state (observer, smoother, ring) on the context stream
  if ((e = hipMemsetAsync(c->st, 0, HW * c->NCOL * Kt * sizeof(float2), c->stream)) != hipSuccess) return bail(e, "memset");
  if ((e = hipMemsetAsync(c->rsm, 0, HW * c->nv * sizeof(float), c->stream)) != hipSuccess) return bail(e, "memset");
  if ((e = hipMemsetAsync(c->ring, 0, HW * c->nring * sizeof(float), c->stream)) != hipSuccess) return bail(e, "memset");
  if ((e = hipMemsetAsync(c->nonfinite, 0, sizeof(unsigned long long), c->stream)) != hipSuccess) return bail(e, "memset");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "sync");
  *out = c;
  return RMDF_OK;
}

static hipEvent_t pooled_event(rmdf_ctx* c) {
  hipEvent_t e = nullptr;
  if (!c->event_pool.empty()) {
    e = c->event_pool.back();
    c->event_pool.pop_back();
  } else {
    hipEventCreate(&e);
  }
  return e;
}
static void timed_begin(rmdf_ctx* c, int which, EventPair* ev) {
  ev->which = -1;
  if (!((c->timing >> which) & 1)) return;
  ev->a = pooled_event(c);
  ev->b = pooled_event(c);
  ev->which = which;
  hipEventRecord(ev->a, c->stream);
}
static void timed_end(rmdf_ctx* c, EventPair* ev) {
  if (ev->which < 0) return;
  hipEventRecord(ev->b, c->stream);
  c->events.push_back(*ev);
}

// The learned network on n feature rows in one kernel (three layers, BF16
// MFMA with FP32 accumulation); list != nullptr also collects the rows whose
// confidence clears the context's threshold.
static hipError_t run_network(rmdf_ctx* c, const unsigned short* feat, int n, float* vc, int* list) {
  return rmdf::launch_mlp_infer(feat, n, c->w1, c->b1, c->w2, c->b2, c->w3, c->b3, vc, c->conf, list, c->stream);
}

rmdf_status rmdf_push_frame(rmdf_ctx* c, const float* frame) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (!frame) return fail(c, RMDF_E_INVAL, "frame is NULL");
  // every check precedes the first launch: a refused push leaves the delay
  // ring, the non-finite counter and the frame count as they were
  if (c->batch_owned) return fail(c, RMDF_E_STATE, "stream owned by a batch: it advances with rmdf_batch_push");
  if (c->vmode == RMDF_VEL_LEARNED && !c->weights_set) return fail(c, RMDF_E_STATE, "learned mode: weights not set");
  const size_t HW = (size_t)c->H * c->W;
  float* slot = c->ring + HW * (size_t)(c->t % c->nring);
  EventPair ev{};
  hipError_t e;
  // row sliding DFT straight from the caller's frame; the same kernel stores
  // the frame (non-finite samples zeroed and counted) into the delay ring
  timed_begin(c, 1, &ev);
  e = rmdf::launch_row(c->MX, frame, c->rs, c->twx, c->H, c->W, slot, c->nonfinite, c->stream,
                       c->temporal == RMDF_TEMPORAL_DIRECT);
  timed_end(c, &ev);
  if (e != hipSuccess) return hip_fail(c, e, "row kernel launch");

  rmdf::PixArgs a = rmdf_internal_pixargs(c);
  a.ring_delayed = (c->t >= c->dt) ? c->ring + HW * (size_t)((c->t - c->dt) % c->nring) : nullptr;
  const int mode = (c->temporal == RMDF_TEMPORAL_DIRECT) ? 5
                   : (c->temporal == RMDF_TEMPORAL_RING) ? 4
                   : (c->vmode == RMDF_VEL_LEARNED) ? 2
                   : (c->vmode == RMDF_VEL_REFINED) ? 3
                   : (c->write_features ? 1 : 0);
  a.tcur = (int)(c->t & 0x3fffffff);
  timed_begin(c, 0, &ev);
  e = (c->variant == 2) ? rmdf::launch_pixel16(a, mode, c->stream)
                        : rmdf::launch_pixel(c->MX, c->MY, c->MZ, a, c->stream);
  timed_end(c, &ev);
  if (e != hipSuccess) return hip_fail(c, e, "pixel kernel launch");
  if (mode == 2) {
    // network on every anchor's features (BF16 MFMA, FP32 accumulate), then
    // the background estimate with the chosen velocity
    // (the network kernel also lists the anchors whose confidence clears
    // the threshold; the finish pass filters those)
    timed_begin(c, 3, &ev);
    e = rmdf::launch_conf_reset(c->conf_list, c->stream);
    if (e == hipSuccess) e = run_network(c, c->feat, c->H * c->W, c->vc, c->conf_list);
    timed_end(c, &ev);
    if (e != hipSuccess) return hip_fail(c, e, "network launch");
    timed_begin(c, 4, &ev);
    e = rmdf::launch_finish16(a, c->vc, c->conf, c->conf_list, c->stream);
    timed_end(c, &ev);
    if (e != hipSuccess) return hip_fail(c, e, "finish kernel launch");
  }
  c->t += 1;
  return RMDF_OK;
}

// Two frames through one pass of the per-pixel kernel (mode 6).
static rmdf_status push_pair(rmdf_ctx* c, const float* f0, const float* f1, float* out0) {
  const size_t HW = (size_t)c->H * c->W;
  auto slot = [&](long long t) { return c->ring + HW * (size_t)(t % c->nring); };
  EventPair ev{};
  hipError_t e;
  // row pass of each frame into its own row spectra (each also stores its
  // frame into its delay-ring slot)
  timed_begin(c, 1, &ev);
  e = rmdf::launch_row(c->MX, f0, c->rs, c->twx, c->H, c->W, slot(c->t), c->nonfinite, c->stream);
  if (e == hipSuccess)
    e = rmdf::launch_row(c->MX, f1, c->rs2, c->twx, c->H, c->W, slot(c->t + 1), c->nonfinite, c->stream);
  timed_end(c, &ev);
  if (e != hipSuccess) return hip_fail(c, e, "row kernel launch");
  rmdf::PixArgs a = rmdf_internal_pixargs(c);
  a.rs2 = c->rs2;
  a.ring_delayed = (c->t >= c->dt) ? slot(c->t - c->dt) : nullptr;
  a.ring_delayed2 = (c->t + 1 >= c->dt) ? slot(c->t + 1 - c->dt) : nullptr;
  a.out_first = out0 ? out0 : c->out_first;
  a.tcur = (int)(c->t & 0x3fffffff);
  timed_begin(c, 0, &ev);
  e = rmdf::launch_pixel16(a, 6, c->stream);
  timed_end(c, &ev);
  if (e != hipSuccess) return hip_fail(c, e, "pixel kernel launch");
  c->t += 2;
  return RMDF_OK;
}

rmdf_status rmdf_push_frames(rmdf_ctx* c, int n, const float* const* frames, float* const* outs) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (n < 1 || !frames) return fail(c, RMDF_E_INVAL, "n must be >= 1 and frames non-NULL");
  for (int i = 0; i < n; ++i)
    if (!frames[i]) return fail(c, RMDF_E_INVAL, "frame is NULL");
  if (c->batch_owned) return fail(c, RMDF_E_STATE, "stream owned by a batch: it advances with rmdf_batch_push");
  if (c->vmode == RMDF_VEL_LEARNED && !c->weights_set) return fail(c, RMDF_E_STATE, "learned mode: weights not set");
  const size_t bytes = (size_t)c->H * c->W * sizeof(float);
  for (int i = 0; i < n;) {
    float* o0 = outs ? outs[i] : nullptr;
    if (pairs_supported(c) && i + 1 < n) {
      const rmdf_status st = push_pair(c, frames[i], frames[i + 1], o0);
      if (st != RMDF_OK) return st;
      float* o1 = outs ? outs[i + 1] : nullptr;
      hipError_t e;
      if (o1 && (e = hipMemcpyAsync(o1, c->out, bytes, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy");
      i += 2;
    } else {
      const rmdf_status st = rmdf_push_frame(c, frames[i]);
      if (st != RMDF_OK) return st;
      hipError_t e;
      if (o0 && (e = hipMemcpyAsync(o0, c->out, bytes, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copy");
      i += 1;
    }
  }
  return RMDF_OK;
}

rmdf_status rmdf_velocity(rmdf_ctx* c, float* vxy, int* idx) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (c->t == 0) return fail(c, RMDF_E_STATE, "no frame pushed yet");
  const size_t HW = (size_t)c->H * c->W;
  hipError_t e;
  if (vxy && (e = hipMemcpyAsync(vxy, c->vxy, HW * sizeof(float2), hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
    return hip_fail(c, e, "velocity copy");
  if (idx && (e = hipMemcpyAsync(idx, c->vidx, HW * sizeof(int), hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
    return hip_fail(c, e, "index copy");
  return RMDF_OK;
}

rmdf_status rmdf_output(rmdf_ctx* c, float* out) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (!out) return fail(c, RMDF_E_INVAL, "out is NULL");
  if (c->t == 0) return fail(c, RMDF_E_STATE, "no frame pushed yet");
  hipError_t e = hipMemcpyAsync(out, c->out, (size_t)c->H * c->W * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "output copy");
  return RMDF_OK;
}

rmdf_status rmdf_frames_pushed(const rmdf_ctx* c, long long* n) {
  if (!c || !n) return RMDF_E_INVAL;
  *n = c->t;
  return RMDF_OK;
}

rmdf_status rmdf_nonfinite_count(rmdf_ctx* c, long long* n) {
  if (!c || !n) return fail(c, RMDF_E_INVAL, "NULL argument");
  unsigned long long v = 0;
  hipError_t e = hipMemcpyAsync(&v, c->nonfinite, sizeof(v), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "counter read");
  *n = (long long)v;
  return RMDF_OK;
}

static int spectrum_layout(const rmdf_ctx* c) {
  return c->temporal != RMDF_TEMPORAL_OBSERVER ? 2 : (c->variant == 2 ? 1 : 0);
}

static rmdf_status spectrum_args(rmdf_ctx* c, int npix, const int* xs, const int* ys, const float* spec) {
  if (npix < 0 || (npix > 0 && (!xs || !ys || !spec))) return fail(c, RMDF_E_INVAL, "bad arguments");
  if (c->t == 0) return fail(c, RMDF_E_STATE, "no frame pushed yet");
  for (int i = 0; i < npix; ++i)
    if (xs[i] < 0 || xs[i] >= c->W || ys[i] < 0 || ys[i] >= c->H) return fail(c, RMDF_E_INVAL, "anchor outside the frame");
  return RMDF_OK;
}

rmdf_status rmdf_spectrum(rmdf_ctx* c, int npix, const int* xs, const int* ys, float* spec) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  rmdf_status st = spectrum_args(c, npix, xs, ys, spec);
  if (st != RMDF_OK || npix == 0) return st;
  // anchor coordinates staged as (x, y) pairs in a device buffer that grows on demand
  std::vector<int> xy(2 * (size_t)npix);
  for (int i = 0; i < npix; ++i) {
    xy[2 * (size_t)i] = xs[i];
    xy[2 * (size_t)i + 1] = ys[i];
  }
  hipError_t e;
  if (npix > c->xy_cap) {
    // the previous buffer is idle (every call ends with a stream synchronisation)
    if (c->xy_scratch) {
      for (auto it = c->allocs.begin(); it != c->allocs.end(); ++it)
        if (*it == static_cast<void*>(c->xy_scratch)) {
          c->allocs.erase(it);
          break;
        }
      hipFree(c->xy_scratch);
      c->bytes -= 2 * (size_t)c->xy_cap * sizeof(int);
      c->xy_scratch = nullptr;
      c->xy_cap = 0;
    }
    if ((e = dalloc(c, &c->xy_scratch, 2 * (size_t)npix)) != hipSuccess) return hip_fail(c, e, "scratch");
    c->xy_cap = npix;
  }
  if ((e = hipMemcpyAsync(c->xy_scratch, xy.data(), xy.size() * sizeof(int), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return hip_fail(c, e, "anchor upload");
  e = rmdf::launch_spectrum(c->MX, c->MY, c->MZ, c->st, c->W, c->xy_scratch, npix, reinterpret_cast<float2*>(spec),
                            spectrum_layout(c), (int)((c->t - 1) & 0x3fffffff), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "spectrum launch");
  // the host array must outlive the copy
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sync");
  return RMDF_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free variant of rmdf_spectrum.  The anchor coordinates go to a
// file-scope device array instead of a buffer the context allocates: xs in
// [0, MAX), ys in [MAX, 2 MAX).  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in symbol): its device
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, and that address is used everywhere.
static __device__ __align__(256) int scratch[2 * RMDF_SPECTRUM_NOALLOC_MAX];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on `device` (looked up on the first call for that
// device, with the device made current for the lookup).
static hipError_t noalloc_scratch(int device, int** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr && g_scratch_err[device] == hipSuccess) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess && p == nullptr) e = hipErrorInvalidSymbol;
    if (e == hipSuccess) g_scratch_ptr[device] = static_cast<int*>(p);
    else g_scratch_err[device] = e;
  }
  *out = g_scratch_ptr[device];
  return g_scratch_ptr[device] ? hipSuccess : g_scratch_err[device];
}

rmdf_status rmdf_spectrum_noalloc(rmdf_ctx* c, int npix, const int* xs, const int* ys, float* spec) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (npix > RMDF_SPECTRUM_NOALLOC_MAX)
    return fail(c, RMDF_E_INVAL, "too many anchors for the allocation-free call (at most RMDF_SPECTRUM_NOALLOC_MAX)");
  rmdf_status st = spectrum_args(c, npix, xs, ys, spec);
  if (st != RMDF_OK || npix == 0) return st;
  int* dev = nullptr;
  hipError_t e = noalloc_scratch(c->device, &dev);
  if (e != hipSuccess) return hip_fail(c, e, "scratch address");
  int* dxs = dev;
  int* dys = dev + RMDF_SPECTRUM_NOALLOC_MAX;
  if ((e = hipMemcpyAsync(dxs, xs, sizeof(int) * npix, hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(dys, ys, sizeof(int) * npix, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return hip_fail(c, e, "anchor upload");
  e = rmdf::launch_spectrum_at(c->MX, c->MY, c->MZ, c->st, c->W, dxs, dys, 1, npix, reinterpret_cast<float2*>(spec),
                               spectrum_layout(c), (int)((c->t - 1) & 0x3fffffff), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "spectrum launch");
  // the caller's host arrays must outlive the copies
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sync");
  return RMDF_OK;
}

rmdf_status rmdf_smoothed_r(rmdf_ctx* c, float* rs) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (!rs) return fail(c, RMDF_E_INVAL, "rs is NULL");
  if (c->t == 0) return fail(c, RMDF_E_STATE, "no frame pushed yet");
  hipError_t e = hipMemcpyAsync(rs, c->rsm, (size_t)c->H * c->W * c->nv * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "copy");
  return RMDF_OK;
}

rmdf_status rmdf_set_timing(rmdf_ctx* c, int on) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  c->timing = on < 0 ? 0x1f : (on & 0x1f);
  return RMDF_OK;
}

rmdf_status rmdf_kernel_time(rmdf_ctx* c, int which, double* ms, long long* launches) {
  if (!c || which < 0 || which > 4 || !ms || !launches) return fail(c, RMDF_E_INVAL, "bad arguments");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sync");
  for (auto& ev : c->events) {
    float t = 0.f;
    hipEventElapsedTime(&t, ev.a, ev.b);
    c->ms[ev.which] += t;
    c->launches[ev.which] += 1;
    c->event_pool.push_back(ev.a);
    c->event_pool.push_back(ev.b);
  }
  c->events.clear();
  *ms = c->ms[which];
  *launches = c->launches[which];
  c->ms[which] = 0;
  c->launches[which] = 0;
  return RMDF_OK;
}

rmdf_status rmdf_mlp_set_weights(rmdf_ctx* c, const float* w, size_t bytes) {
  if (!c || !w) return fail(c, RMDF_E_INVAL, "NULL argument");
  if (c->vmode != RMDF_VEL_LEARNED) return fail(c, RMDF_E_STATE, "context is not in learned mode");
  const size_t n1 = 128 * 1152, n2 = 64 * 128;
  const size_t total = n1 + 128 + n2 + 64 + 192 + 3;
  if (bytes != total * sizeof(float)) return fail(c, RMDF_E_INVAL, "weight blob has the wrong size");
  for (size_t i = 0; i < total; ++i)
    if (!std::isfinite(w[i])) return fail(c, RMDF_E_INVAL, "non-finite weight");
  auto bf = [](float f) {
    unsigned int u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
  };
  std::vector<unsigned short> w1(n1), w2(n2);
  for (int col = 0; col < 128; ++col)
    for (int k = 0; k < 1152; ++k) w1[rmdf::mlp_w1_packed_index(col, k)] = bf(w[(size_t)col * 1152 + k]);
  const float* p = w + n1;
  const float* b1 = p; p += 128;
  for (size_t i = 0; i < n2; ++i) w2[i] = bf(p[i]);
  p += n2;
  const float* b2 = p; p += 64;
  const float* w3 = p; p += 192;
  const float* b3 = p;
  // enqueued on the context stream, so the upload is ordered after every push
  // already queued there (they read the previous weights) and before the next;
  // the host staging arrays must outlive the copies, hence the synchronisation
  hipError_t e;
  auto up = [&](void* dst, const void* src, size_t n) {
    return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->stream);
  };
  if ((e = up(c->w1, w1.data(), n1 * 2)) != hipSuccess || (e = up(c->w2, w2.data(), n2 * 2)) != hipSuccess ||
      (e = up(c->b1, b1, 128 * 4)) != hipSuccess || (e = up(c->b2, b2, 64 * 4)) != hipSuccess ||
      (e = up(c->w3, w3, 192 * 4)) != hipSuccess || (e = up(c->b3, b3, 3 * 4)) != hipSuccess)
    return hip_fail(c, e, "weight upload");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "weight upload");
  c->weights_set = true;
  return RMDF_OK;
}

rmdf_status rmdf_features(rmdf_ctx* c, void* feat_dev) {
  if (!c || !feat_dev) return fail(c, RMDF_E_INVAL, "NULL argument");
  if (!c->feat) return fail(c, RMDF_E_STATE, "context computes no features");
  if (c->t == 0) return fail(c, RMDF_E_STATE, "no frame pushed yet");
  hipError_t e = hipMemcpyAsync(feat_dev, c->feat, (size_t)c->H * c->W * 1152 * 2, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "copy");
  return RMDF_OK;
}

rmdf_status rmdf_learned_output(rmdf_ctx* c, float* vc_dev) {
  if (!c || !vc_dev) return fail(c, RMDF_E_INVAL, "NULL argument");
  if (!c->vc) return fail(c, RMDF_E_STATE, "context is not in learned mode");
  if (c->t == 0) return fail(c, RMDF_E_STATE, "no frame pushed yet");
  hipError_t e = hipMemcpyAsync(vc_dev, c->vc, (size_t)c->H * c->W * 3 * 4, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "copy");
  return RMDF_OK;
}

rmdf_status rmdf_learned_network(rmdf_ctx* c, const void* feat_dev, int n, float* vc_dev) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (!feat_dev || !vc_dev || n < 1) return fail(c, RMDF_E_INVAL, "bad arguments");
  if (c->vmode != RMDF_VEL_LEARNED) return fail(c, RMDF_E_STATE, "context is not in learned mode");
  if (!c->weights_set) return fail(c, RMDF_E_STATE, "learned mode: weights not set");
  if (reinterpret_cast<uintptr_t>(feat_dev) & 15) return fail(c, RMDF_E_INVAL, "features not 16-byte aligned");
  const hipError_t e = run_network(c, static_cast<const unsigned short*>(feat_dev), n, vc_dev, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "network launch");
  return RMDF_OK;
}

// ---------------------------------------------------------------------------
// Saved states: a 128-byte header, then the sections below, each starting on a
// 256-byte boundary.
namespace {
struct StateHeader {
  char magic[8];                   // "RMDFST1"
  unsigned int version, header_bytes;
  int H, W, MX, MY, MZ, nvx, nvy, variant, temporal, nring, dt, reserved;
  long long t;                     // frames pushed
  unsigned long long nonfinite;    // non-finite samples replaced so far
  unsigned long long param_hash;
  unsigned char pad[40];
};
static_assert(sizeof(StateHeader) == 128, "state header layout");
constexpr char kStateMagic[8] = {'R', 'M', 'D', 'F', 'S', 'T', '1', 0};
constexpr size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

struct Section {
  void* dev;
  size_t bytes;
};
}  // namespace

// The recursive state: observer (or 2-D spectrum ring), smoothed R, delay
// ring; then the latest readouts.
static std::vector<Section> state_sections(const rmdf_ctx* c) {
  const size_t HW = (size_t)c->H * c->W;
  return {{c->st, HW * c->NCOL * c->MZ * sizeof(float2)},
          {c->rsm, HW * c->nv * sizeof(float)},
          {c->ring, HW * c->nring * sizeof(float)},
          {c->out, HW * sizeof(float)},
          {c->vxy, HW * sizeof(float2)},
          {c->vidx, HW * sizeof(int)}};
}

static size_t state_size(const rmdf_ctx* c) {
  size_t n = sizeof(StateHeader);
  for (const Section& sec : state_sections(c)) n = align256(n) + sec.bytes;
  return n;
}

static StateHeader state_header(const rmdf_ctx* c) {
  StateHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kStateMagic, sizeof h.magic);
  h.version = 1;
  h.header_bytes = sizeof(StateHeader);
  h.H = c->H; h.W = c->W; h.MX = c->MX; h.MY = c->MY; h.MZ = c->MZ;
  h.nvx = c->nvx; h.nvy = c->nvy; h.variant = c->variant; h.temporal = c->temporal;
  h.nring = c->nring; h.dt = c->dt;
  h.param_hash = c->param_hash;
  h.t = c->t;
  return h;
}

rmdf_status rmdf_state_bytes(const rmdf_ctx* c, size_t* bytes) {
  if (!c || !bytes) return RMDF_E_INVAL;
  *bytes = state_size(c);
  return RMDF_OK;
}

rmdf_status rmdf_save_state(rmdf_ctx* c, void* buf, size_t bytes) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (!buf) return fail(c, RMDF_E_INVAL, "buffer is NULL");
  if (bytes < state_size(c)) return fail(c, RMDF_E_INVAL, "buffer smaller than rmdf_state_bytes");
  StateHeader h = state_header(c);
  hipError_t e = hipMemcpyAsync(&h.nonfinite, c->nonfinite, sizeof h.nonfinite, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "counter read");
  char* dst = static_cast<char*>(buf);
  if ((e = hipMemcpyAsync(dst, &h, sizeof h, hipMemcpyDefault, c->stream)) != hipSuccess) return hip_fail(c, e, "save");
  size_t off = sizeof h;
  for (const Section& sec : state_sections(c)) {
    off = align256(off);
    if ((e = hipMemcpyAsync(dst + off, sec.dev, sec.bytes, hipMemcpyDefault, c->stream)) != hipSuccess)
      return hip_fail(c, e, "save");
    off += sec.bytes;
  }
  // the header lives on this stack frame: wait for the copies
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "save");
  return RMDF_OK;
}

rmdf_status rmdf_load_state(rmdf_ctx* c, const void* buf, size_t bytes) {
  if (!c) return fail(nullptr, RMDF_E_INVAL, "ctx is NULL");
  if (!buf) return fail(c, RMDF_E_INVAL, "buffer is NULL");
  if (c->batch_owned) return fail(c, RMDF_E_STATE, "stream owned by a batch: its frame count lives in the batch");
  if (bytes < sizeof(StateHeader)) return fail(c, RMDF_E_INVAL, "buffer too small for a saved state");
  StateHeader h;
  hipError_t e = hipMemcpyAsync(&h, buf, sizeof h, hipMemcpyDefault, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "header read");
  const StateHeader mine = state_header(c);
  if (std::memcmp(h.magic, kStateMagic, sizeof h.magic) != 0 || h.version != 1 || h.header_bytes != sizeof h)
    return fail(c, RMDF_E_INVAL, "not a saved rmdf state");
  if (h.H != mine.H || h.W != mine.W || h.MX != mine.MX || h.MY != mine.MY || h.MZ != mine.MZ ||
      h.nvx != mine.nvx || h.nvy != mine.nvy || h.variant != mine.variant || h.temporal != mine.temporal ||
      h.nring != mine.nring || h.dt != mine.dt)
    return fail(c, RMDF_E_INVAL, "saved state belongs to a context of another shape");
  if (h.param_hash != mine.param_hash)
    return fail(c, RMDF_E_INVAL, "saved state belongs to a context with another grid or parameters");
  if (h.t < 0) return fail(c, RMDF_E_INVAL, "saved state has a negative frame count");
  if (bytes < state_size(c)) return fail(c, RMDF_E_INVAL, "buffer shorter than the saved state");
  const char* src = static_cast<const char*>(buf);
  size_t off = sizeof h;
  for (const Section& sec : state_sections(c)) {
    off = align256(off);
    if ((e = hipMemcpyAsync(sec.dev, src + off, sec.bytes, hipMemcpyDefault, c->stream)) != hipSuccess)
      return hip_fail(c, e, "load");
    off += sec.bytes;
  }
  if ((e = hipMemcpyAsync(c->nonfinite, &h.nonfinite, sizeof h.nonfinite, hipMemcpyHostToDevice, c->stream)) !=
      hipSuccess)
    return hip_fail(c, e, "load");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "load");
  c->t = h.t;
  return RMDF_OK;
}

rmdf_status rmdf_kernel_variant(const rmdf_ctx* c, int* variant) {
  if (!c || !variant) return RMDF_E_INVAL;
  *variant = c->variant;
  return RMDF_OK;
}

rmdf_status rmdf_tile_rows(const rmdf_ctx* c, int* tile_rows) {
  if (!c || !tile_rows) return RMDF_E_INVAL;
  *tile_rows = c->TY;
  return RMDF_OK;
}

rmdf_status rmdf_coeff_lattice(const rmdf_ctx* c, int* lattice_q) {
  if (!c || !lattice_q) return RMDF_E_INVAL;
  *lattice_q = (c->variant == 2 && c->vmode != RMDF_VEL_REFINED) ? c->lat_q : 0;
  return RMDF_OK;
}

rmdf_status rmdf_device_bytes(const rmdf_ctx* c, size_t* bytes) {
  if (!c || !bytes) return RMDF_E_INVAL;
  *bytes = c->bytes;
  return RMDF_OK;
}

rmdf_status rmdf_destroy(rmdf_ctx* c) {
  if (!c) return RMDF_OK;
  if (c->stream) hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return RMDF_OK;
}

const char* rmdf_last_error(const rmdf_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
