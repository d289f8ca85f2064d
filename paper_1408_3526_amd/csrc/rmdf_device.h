// rmdf_device.h - device-side building blocks of the recursive
// multidimensional prediction-error filter (Kennedy, arXiv:1408.3526): complex
// helpers, the row sliding-DFT chunk and the generic per-pixel work tile.
// Included by every translation unit that launches them (no relocatable
// device code is used).
#pragma once
#include <hip/hip_runtime.h>

#include "rmdf_kernels.h"
#include "rmdf_refine.h"
#include "rmdf_wave.h"

namespace rmdf {

static __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
static __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
static __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
static __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
static __device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Workgroup barrier that orders LDS only: outstanding global loads (the
// prefetch of the next row's observer state) stay in flight across it.
static __device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int MX>
struct RowShape {
  static constexpr int NP = (MX % 2 == 0) ? MX / 2 : (MX + 1) / 2;
  static constexpr size_t SMEM = sizeof(float) * (MX + RCX) + sizeof(float2) * (NP * RCX + MX);
};

// One (row y, chunk of RCX columns starting at x0).  Non-finite samples are
// read as 0; when `nonfinite` is given, those of the chunk's own columns are
// counted; when `copy_to` is given, the chunk's own columns are stored there
// (non-finite ones as 0): the frame's copy into the delay ring.
// DIRECT: every output is the direct Mx-term DFT sum of its window (no comb,
// no resonator): the non-recursive form of the same row spectrum.
template <int MX, bool DIRECT = false>
static __device__ void row_chunk(const float* __restrict__ f, float2* __restrict__ rs, const float2* __restrict__ twx,
                          int H, int W, int y, int x0, char* smem, unsigned long long* nonfinite,
                          float* __restrict__ copy_to = nullptr) {
  constexpr int NP = RowShape<MX>::NP;
  constexpr int NSEG = RCX / RSEG;
  constexpr bool EVEN = (MX % 2 == 0);
  float* s_in = reinterpret_cast<float*>(smem);                          // [MX + RCX]
  float2* s_out = reinterpret_cast<float2*>(smem + sizeof(float) * (MX + RCX));   // [NP][RCX]
  float2* s_tw = s_out + NP * RCX;                                       // [MX]
  const float* row = f + (size_t)y * W;
  int bad = 0;
  for (int i = threadIdx.x; i < MX + RCX; i += blockDim.x) {
    const int xx = x0 - MX + i;
    float v = (xx >= 0 && xx < W) ? row[xx] : 0.0f;
    if (!isfinite(v)) {
      v = 0.0f;
      bad += (i >= MX) ? 1 : 0;     // count the chunk's own columns only
    }
    s_in[i] = v;
    if (copy_to != nullptr && i >= MX && xx < W) copy_to[(size_t)y * W + xx] = v;
  }
  for (int i = threadIdx.x; i < MX; i += blockDim.x) s_tw[i] = twx[i];
  if (nonfinite) {
    // the wavefront's count, reduced only where it has non-finite samples
    if (__ballot(bad != 0)) {
      int tot = bad;
      for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
      if ((threadIdx.x & 63) == 0) atomicAdd(nonfinite, (unsigned long long)tot);
    }
  }
  __syncthreads();
  const float inv = rsqrtf((float)MX);
  if (DIRECT && threadIdx.x < NP * NSEG) {
    // A(kx; x) = sum_m w^(kx m) I(x - m), m = 0 .. Mx - 1, for each column
    const int p = threadIdx.x / NSEG, sg = threadIdx.x % NSEG;
    const int xs = sg * RSEG;
    for (int i = 0; i < RSEG; ++i) {
      const int xi = xs + i;
      if (p == 0) {
        float a0 = 0.f, ah = 0.f;
        for (int m = 0; m < MX; ++m) {
          const float v = s_in[MX + xi - m];
          a0 += v;
          ah += (m & 1) ? -v : v;
        }
        s_out[xi] = EVEN ? make_float2(a0 * inv, ah * inv) : make_float2(a0 * inv, 0.f);
      } else {
        float2 acc = make_float2(0.f, 0.f);
        for (int m = 0; m < MX; ++m) {
          const float v = s_in[MX + xi - m];
          const float2 w = s_tw[(p * m) % MX];
          acc.x += w.x * v;
          acc.y += w.y * v;
        }
        s_out[p * RCX + xi] = cscale(acc, inv);
      }
    }
  } else if (threadIdx.x < NP * NSEG) {
    const int p = threadIdx.x / NSEG, sg = threadIdx.x % NSEG;
    const int xs = sg * RSEG;             // segment start relative to x0
    if (p == 0) {
      // kx = 0 (pole 1) and, for even Mx, kx = Mx/2 (pole -1): real resonators
      float a0 = 0.f, ah = 0.f;
      for (int m = 0; m < MX; ++m) {
        const float v = s_in[MX + xs - 1 - m];
        a0 += v;
        ah += (m & 1) ? -v : v;
      }
      for (int i = 0; i < RSEG; ++i) {
        const int xi = xs + i;
        const float comb = s_in[MX + xi] - s_in[xi];
        a0 = a0 + comb;
        ah = -ah + comb;
        s_out[xi] = EVEN ? make_float2(a0 * inv, ah * inv) : make_float2(a0 * inv, 0.f);
      }
    } else {
      float2 acc = make_float2(0.f, 0.f);
      for (int m = 0; m < MX; ++m) {
        const float v = s_in[MX + xs - 1 - m];
        const float2 w = s_tw[(p * m) % MX];
        acc.x += w.x * v;
        acc.y += w.y * v;
      }
      const float2 w1 = s_tw[p];
      for (int i = 0; i < RSEG; ++i) {
        const int xi = xs + i;
        const float comb = s_in[MX + xi] - s_in[xi];
        acc = cmul(w1, acc);
        acc.x += comb;
        s_out[p * RCX + xi] = cscale(acc, inv);
      }
    }
  }
  __syncthreads();
  // row spectra layout [y][x][plane]: the planes of a pixel are adjacent, so
  // the per-pixel kernels read one contiguous run per row and workgroup
  for (int i = threadIdx.x; i < NP * RCX; i += blockDim.x) {
    const int xi = i / NP, p = i % NP;
    if (x0 + xi < W) rs[((size_t)y * W + x0 + xi) * NP + p] = s_out[p * RCX + xi];
  }
}

// ---------------------------------------------------------------------------
// Per-pixel kernel.
template <int MX, int MY, int MZ>
struct Shape {
  static constexpr bool EVEN = (MX % 2 == 0);
  static constexpr int NP = EVEN ? MX / 2 : (MX + 1) / 2;   // stored kx planes
  static constexpr int NXH = MX / 2 + 1;                    // kx = 0 .. Mx/2
  static constexpr int NCOL = NP * MY;                      // (plane, ky) columns
  static constexpr int NCOLP = NCOL <= 32 ? 32 : (NCOL <= 64 ? 64 : (NCOL <= 128 ? 128 : 256));
  static constexpr int PPB = 256 / NCOLP;                   // pixels per block row-step
  static constexpr int A_ELEMS = PPB * NCOL * MZ;           // Hann staging (float2)
  static constexpr int QT_ELEMS = PPB * NXH * (MY + NVY_MAX);
  static constexpr int U_ELEMS = A_ELEMS > QT_ELEMS ? A_ELEMS : QT_ELEMS;
  static constexpr int TAB_ELEMS = NVY_MAX * MY + NVX_MAX * NXH;  // tau_y and tau_x, staged per tile
  static constexpr size_t SMEM = sizeof(float2) * (U_ELEMS + A_ELEMS + 2 * MZ + MY + TAB_ELEMS) +
                                 (sizeof(float) + sizeof(int)) * 256;
};


// Eq. (8) at bin (kx, ky, kz) for a continuous velocity (the spatial Dirichlet
// factors select kx' = kx, ky' = ky at the bins), times sqrt(Mz) since the
// state holds S / sqrt(Mz):
//   D_Mz(kz/Mz + phi) / sqrt(Mx My) * exp(j pi [-2(kx m'x/Mx + ky m'y/My)
//   + 2 phi (m't - Dz) - 2 kz Dz/Mz]),  phi = vx kx/Mx + vy ky/My.
template <int MX, int MY, int MZ>
static __device__ __forceinline__ float2 coeff_at(int kx, int ky, int kz, float vx, float vy, int dx, int dy, int dt) {
  const float Dz = 0.5f * (MZ - 1);
  const float phi = vx * kx * (1.0f / MX) + vy * ky * (1.0f / MY);
  const float w = kz * (1.0f / MZ) + phi;
  const float rw = rintf(w);
  float D;
  if (fabsf(w - rw) < 1e-5f) D = (((int)rw * (MZ - 1)) & 1) ? -1.f : 1.f;
  else D = sinpif(MZ * w) / (MZ * sinpif(w));
  const float ph = -2.f * (kx * (float)dx / MX + ky * (float)dy / MY) + 2.f * phi * (dt - Dz) - 2.f * kz * Dz / MZ;
  float sn, cs;
  sincospif(ph, &sn, &cs);
  const float g = D * (1.0f / sqrtf((float)(MX * MY)));
  return make_float2(g * cs, g * sn);
}

// One work tile: PPB adjacent anchor columns starting at xb*PPB, rows
// [yb*TY, yb*TY + TY).  All 256 threads of the block must call it.
template <int MX, int MY, int MZ>
static __device__ __forceinline__ void pixel_tile(const PixArgs& a, const float* ring_delayed, int xb, int yb, char* smem) {
  using SH = Shape<MX, MY, MZ>;
  constexpr int NP = SH::NP, NXH = SH::NXH, NCOL = SH::NCOL, NCOLP = SH::NCOLP, PPB = SH::PPB;
  constexpr bool EVEN = SH::EVEN;

  float2* s_u = reinterpret_cast<float2*>(smem);  // Hann-z stage, later Q and T
  float2* s_b = s_u + SH::U_ELEMS;                 // Hann-y stage
  float2* s_twz = s_b + SH::A_ELEMS;
  float2* s_twA = s_twz + MZ;
  float2* s_twy = s_twA + MZ;
  float2* s_tauy = s_twy + MY;                   // [nvy][MY]
  float2* s_taux = s_tauy + NVY_MAX * MY;        // [nvx][NXH]
  float* s_rv = reinterpret_cast<float*>(s_taux + NVX_MAX * NXH);
  int* s_ri = reinterpret_cast<int*>(s_rv + 256);

  const int tid = threadIdx.x;
  const int ps = tid / NCOLP, c = tid % NCOLP;
  const int x = xb * PPB + ps;
  const bool px_ok = x < a.W;
  const bool col_ok = px_ok && c < NCOL;
  const int p = c / MY, ky = c % MY;
  const int y0 = yb * a.TY;
  const int y1 = min(a.H, y0 + a.TY);

  for (int i = tid; i < MZ; i += 256) { s_twz[i] = a.twz[i]; s_twA[i] = a.twA[i]; }
  for (int i = tid; i < MY; i += 256) s_twy[i] = a.twy[i];
  // the stage B and C weight tables too: read there once per candidate and
  // row, from LDS they add no global-load latency to every row's flow
  for (int i = tid; i < a.nvy * MY; i += 256) s_tauy[i] = a.tauy[i];
  for (int i = tid; i < a.nvx * NXH; i += 256) s_taux[i] = a.taux[i];
  __syncthreads();

  float2* s_a = s_u;                                   // [PPB][NCOL][MZ]
  float2* s_q = s_u;                                   // [PPB][NXH][MY]
  float2* s_t = s_u + PPB * NXH * MY;                  // [PPB][NXH][NVY_MAX]
  const int nvx = a.nvx, nvy = a.nvy, nv = a.nv;

  // Column sliding DFT: seed with the direct DFT of the My rows above y0
  // (rows above the frame count as zero).  All My loads are issued before the
  // sum, so a tile start costs one memory latency, not My of them.
  float2 acol = make_float2(0.f, 0.f);
  if (col_ok) {
    float2 v[MY];
#pragma unroll
    for (int m = 0; m < MY; ++m) {
      const int yy = y0 - 1 - m;
      v[m] = (yy >= 0) ? a.rs[((size_t)yy * a.W + x) * NP + p] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < MY; ++m) acol = cadd(acol, cmul(s_twy[(ky * m) % MY], v[m]));
  }
  const float2 wy = s_twy[ky % MY];

  float2 X[MZ];
  if (col_ok && y0 < y1) {
    const float2* src = a.st + (((size_t)y0 * a.W + x) * NCOL + c) * MZ;
#pragma unroll
    for (int k = 0; k < MZ; ++k) X[k] = src[k];
  } else {
#pragma unroll
    for (int k = 0; k < MZ; ++k) X[k] = make_float2(0.f, 0.f);
  }

  for (int y = y0; y < y1; ++y) {
    const size_t pix = (size_t)y * a.W + x;
    // ---- column sliding DFT: comb on the row spectra, resonator w_y^ky
    if (col_ok) {
      float2 in = a.rs[((size_t)y * a.W + x) * NP + p];
      if (y >= MY) in = csub(in, a.rs[((size_t)(y - MY) * a.W + x) * NP + p]);
      acol = cadd(cmul(wy, acol), in);
    }
    const float2 s2 = cscale(acol, a.inv_sqrt_my);

    // ---- temporal deadbeat observer: prior = rotate(posterior), innovation
    // e = input - sum(prior), posterior = prior + e / Mz
    if (col_ok) {
      float2 sum = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < MZ; ++k) {
        X[k] = cmul(s_twz[k], X[k]);
        sum = cadd(sum, X[k]);
      }
      const float2 e = cscale(csub(s2, sum), 1.0f / MZ);
#pragma unroll
      for (int k = 0; k < MZ; ++k) X[k] = cadd(X[k], e);
      float2* dst = a.st + (pix * NCOL + c) * MZ;
#pragma unroll
      for (int k = 0; k < MZ; ++k) dst[k] = X[k];
    }
    // prefetch the next row's state (in flight during the flow stages)
    float2 Xn[MZ];
    if (col_ok && y + 1 < y1) {
      const float2* src = a.st + ((pix + a.W) * NCOL + c) * MZ;
#pragma unroll
      for (int k = 0; k < MZ; ++k) Xn[k] = src[k];
    } else {
#pragma unroll
      for (int k = 0; k < MZ; ++k) Xn[k] = make_float2(0.f, 0.f);
    }

    // ---- high-pass (drop kx = ky = 0 for every kz) and Hann along kz.
    // Hann along an axis is Y(k) = (2X(k) - X(k-1) - X(k+1)) / 4; the 1/4 per
    // axis is folded into the stage-A weights.
    lds_barrier();     // the previous row's stage C has finished reading s_u
    if (col_ok) {
      float2 V[MZ];
#pragma unroll
      for (int k = 0; k < MZ; ++k) V[k] = X[k];
      if (p == 0 && ky == 0) {
        if (EVEN) {
          // packed plane holds S(0) + j S(Mx/2); remove the S(0) part only:
          // S(0)(0, kz) = (C(kz) + conj C(-kz)) / 2
#pragma unroll
          for (int k = 0; k < MZ; ++k) {
            const float2 cm = X[(MZ - k) % MZ];
            V[k] = make_float2(0.5f * (X[k].x - cm.x), 0.5f * (X[k].y + cm.y));
          }
        } else {
#pragma unroll
          for (int k = 0; k < MZ; ++k) V[k] = make_float2(0.f, 0.f);
        }
      }
      float2* dst = s_a + (ps * NCOL + c) * MZ;
#pragma unroll
      for (int k = 0; k < MZ; ++k) {
        const float2 l = V[(k + MZ - 1) % MZ], r = V[(k + 1) % MZ];
        dst[k] = make_float2(2.f * V[k].x - l.x - r.x, 2.f * V[k].y - l.y - r.y);
      }
    }
    lds_barrier();
    // ---- Hann along ky
    float2 Hy[MZ];
    if (col_ok) {
      const float2* cur = s_a + (ps * NCOL + c) * MZ;
      const float2* lo = s_a + (ps * NCOL + p * MY + (ky + MY - 1) % MY) * MZ;
      const float2* hi = s_a + (ps * NCOL + p * MY + (ky + 1) % MY) * MZ;
#pragma unroll
      for (int k = 0; k < MZ; ++k) {
        const float2 v = cur[k], l = lo[k], r = hi[k];
        Hy[k] = make_float2(2.f * v.x - l.x - r.x, 2.f * v.y - l.y - r.y);
      }
    }
    lds_barrier();     // everyone has read s_a (s_u is reused for Q below)
    if (col_ok) {
      float2* dst = s_b + (ps * NCOL + c) * MZ;
#pragma unroll
      for (int k = 0; k < MZ; ++k) dst[k] = Hy[k];
    }
    lds_barrier();

    // ---- Hann along kx, power spectrum (eq. 9), stage A of eq. (10):
    // Q(kx, ky) = sum_kz P(k) w_z^kz (l_z = 1), kx in [0, Mx/2]
    if (col_ok) {
      const float2* B = s_b + ps * NCOL * MZ;
      // y,z-windowed spectrum at any kx in [0, Mx) from the stored half
      auto Vk = [&](int kx, int kyy, int kz) -> float2 {
        bool cj = false;
        if (2 * kx > MX) { kx = MX - kx; kyy = (MY - kyy) % MY; kz = (MZ - kz) % MZ; cj = true; }
        float2 r;
        if (kx == 0 || (EVEN && 2 * kx == MX)) {
          const float2 u = B[kyy * MZ + kz];
          if (!EVEN) {
            r = u;
          } else {
            const float2 w = B[((MY - kyy) % MY) * MZ + (MZ - kz) % MZ];
            if (kx == 0) r = make_float2(0.5f * (u.x + w.x), 0.5f * (u.y - w.y));
            else         r = make_float2(0.5f * (u.y + w.y), -0.5f * (u.x - w.x));
          }
        } else {
          r = B[(kx * MY + kyy) * MZ + kz];
        }
        return cj ? cconj(r) : r;
      };
      const int nk = (EVEN && p == 0) ? 2 : 1;
      for (int j = 0; j < nk; ++j) {
        const int kx = (j == 0) ? p : MX / 2;
        float2 q = make_float2(0.f, 0.f);
#pragma unroll
        for (int kz = 0; kz < MZ; ++kz) {
          const float2 v = Vk(kx, ky, kz);
          const float2 l = Vk((kx + MX - 1) % MX, ky, kz);
          const float2 r = Vk((kx + 1) % MX, ky, kz);
          const float hx = 2.f * v.x - l.x - r.x, hy = 2.f * v.y - l.y - r.y;
          const float P = hx * hx + hy * hy;
          q.x += P * s_twA[kz].x;
          q.y += P * s_twA[kz].y;
        }
        s_q[(ps * NXH + kx) * MY + ky] = q;
      }
    }
    lds_barrier();

    // ---- stage B: T(kx, iy) = sum_ky Q(kx, ky) tau_y(ky, l_y[iy])
    for (int w = c; w < NXH * nvy; w += NCOLP) {
      const int kx = w / nvy, iy = w % nvy;
      const float2* Q = s_q + (ps * NXH + kx) * MY;
      const float2* ty = s_tauy + iy * MY;
      float2 t = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < MY; ++k) t = cadd(t, cmul(Q[k], ty[k]));
      s_t[(ps * NXH + kx) * NVY_MAX + iy] = t;
    }
    lds_barrier();

    // ---- stage C: R(ix, iy) = sum_kx w(kx) Re[T(kx, iy) tau_x(kx, l_x[ix])],
    // first-order smoothing, running argmax
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int w = c; w < nv; w += NCOLP) {
      const int ix = w % nvx, iy = w / nvx;
      const float2* tx = s_taux + ix * NXH;
      float r = 0.f;
#pragma unroll
      for (int kx = 0; kx < NXH; ++kx) {
        const float2 t = s_t[(ps * NXH + kx) * NVY_MAX + iy];
        r += t.x * tx[kx].x - t.y * tx[kx].y;
      }
      if (px_ok) {
        float* rp = a.rsm + pix * nv + w;
        const float sm = (1.f - a.alpha) * r + a.alpha * (*rp);
        *rp = sm;
        amax_merge(bv, bi, sm, w);
      }
    }
    // reduce (value, index) over the pixel's NCOLP threads (within the
    // wavefront by DPP and lane reads, across wavefronts through LDS)
    group_amax<(NCOLP < 64 ? NCOLP : 64)>(bv, bi);
    if (NCOLP > 64) {
      s_rv[tid] = bv;
      s_ri[tid] = bi;
      lds_barrier();
      for (int wv = 1; wv < NCOLP / 64; ++wv) amax_merge(bv, bi, s_rv[(tid ^ (wv * 64))], s_ri[(tid ^ (wv * 64))]);
      lds_barrier();
    }
    const int istar = (bi < nv) ? bi : 0;   // no finite candidate: fall back to index 0

    // ---- velocity mode 3: refine the peak between grid points, from the
    // smoothed R this row has just stored (the barrier makes the workgroup's
    // global stores visible to all of its threads)
    float2 vref = make_float2(0.f, 0.f);
    if (a.vmode == 3) {
      __syncthreads();
      if (px_ok) {
        const float* rp = a.rsm + pix * nv;
        vref = refine_peak(a.gx, a.gy, nvx, nvy, istar, rp[istar], [&](int w) { return rp[w]; });
      }
    }

    // ---- background estimate (eq. 4) with the coefficients of the chosen
    // velocity (eq. 8 at the bins; Hermitian weights folded into the table, or
    // evaluated here for the refined velocity)
    const int hsel = (a.vmode == 2) ? nv : istar;
    float acc = 0.f;
    if (col_ok && p <= a.bx) {
      const int kyc = (2 * ky <= MY) ? ky : ky - MY;
      if (kyc >= -a.by && kyc <= a.by) {
        if (a.vmode == 3) {
          const float wgt = (p == 0) ? 1.f : 2.f;
#pragma unroll
          for (int kz = 0; kz < MZ; ++kz) {
            const float2 h = coeff_at<MX, MY, MZ>(p, kyc, kz, vref.x, vref.y, a.dx, a.dy, a.dt);
            acc += wgt * (h.x * X[kz].x - h.y * X[kz].y);
          }
        } else {
          const float2* h = a.htab + (((size_t)hsel * (a.bx + 1) + p) * (2 * a.by + 1) + (kyc + a.by)) * MZ;
#pragma unroll
          for (int kz = 0; kz < MZ; ++kz) acc += h[kz].x * X[kz].x - h[kz].y * X[kz].y;
        }
      }
    }
    acc = group_sum<(NCOLP < 64 ? NCOLP : 64)>(acc);
    if (NCOLP > 64) {
      s_rv[tid] = acc;
      lds_barrier();
      float tot = 0.f;
      for (int wv = 0; wv < NCOLP / 64; ++wv) tot += s_rv[(ps * NCOLP) + wv * 64];
      acc = tot;
      lds_barrier();
    }
    if (px_ok && c == 0) {
      const int xs = x - a.dx, ys = y - a.dy;
      float idel = (ring_delayed != nullptr && xs >= 0 && ys >= 0) ? ring_delayed[(size_t)ys * a.W + xs] : 0.f;
      if (!isfinite(idel)) idel = 0.f;
      a.out[pix] = idel - acc;
      if (a.vmode == 2) {
        a.vxy[pix] = make_float2(a.fvx, a.fvy);
        a.vidx[pix] = -1;
      } else {
        a.vxy[pix] = (a.vmode == 3) ? vref : make_float2(a.gx[istar % nvx], a.gy[istar / nvx]);
        a.vidx[pix] = istar;
      }
    }
#pragma unroll
    for (int k = 0; k < MZ; ++k) X[k] = Xn[k];
  }
}

}  // namespace rmdf
