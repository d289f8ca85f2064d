// rmdf_kernels.hip - gfx950 kernels of the recursive multidimensional
// prediction-error filter (Kennedy, arXiv:1408.3526).
//
// Per frame (all on one stream):
//   k_ingest  : frame -> delay ring slot, non-finite samples -> 0 (counted)
//   k_row     : row sliding DFT (comb x(n) - x(n-M) into resonators w^k,
//               Sec. 1, eq. 6-7) -> row spectra rs[plane][y][x]
//   k_pixel   : per anchor (x, y): column sliding DFT, temporal deadbeat
//               observer (state streamed once), high-pass + Hann + power
//               spectrum (eq. 9), autocorrelation on the candidate grid at
//               l_z = 1 (eq. 10), first-order smoothing, argmax, background
//               estimate (eq. 4) with the velocity-tuned coefficients (eq. 8),
//               prediction error (eq. 1).
//
// Spectra of a real input are Hermitian, so only kx in [0, Mx/2] is kept.
// For even Mx the two real-input planes kx = 0 and kx = Mx/2 are packed into
// one complex plane C = S(0) + j S(Mx/2) (every stage before the high-pass is
// linear with identical coefficients for both), giving Mx/2 planes of My x Mz
// complex numbers: exactly Mx*My*Mz reals of observer state per pixel.  For odd
// Mx the kx = 0 plane is stored as is ((Mx+1)/2 planes).
#include <hip/hip_runtime.h>

#include "rmdf_kernels.h"

namespace rmdf {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Workgroup barrier that orders LDS only: outstanding global loads (the
// prefetch of the next row's observer state) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Ingest: copy the caller's frame into the delay ring, zero non-finite values.
__global__ void __launch_bounds__(256) k_ingest(const float* __restrict__ in, float* __restrict__ ring_slot,
                                                long long n, unsigned long long* __restrict__ nonfinite) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) {
    float v = in[i];
    if (!isfinite(v)) { v = 0.0f; bad = 1; }
    ring_slot[i] = v;
  }
  // one atomic per wave that saw a non-finite sample
  unsigned long long m = __ballot(bad);
  if (m && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(nonfinite, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------------------
// Row sliding DFT.  Block = (row y, chunk of RCX columns).  Each (plane,
// segment) thread seeds its resonators with the direct DFT of the Mx samples
// before the segment, then runs the comb/resonator recursion across RSEG
// columns; results are staged in LDS and written coalesced.
template <int MX>
__global__ void __launch_bounds__(256) k_row(const float* __restrict__ f, float2* __restrict__ rs,
                                             const float2* __restrict__ twx, int H, int W) {
  constexpr int NP = (MX % 2 == 0) ? MX / 2 : (MX + 1) / 2;
  constexpr int NSEG = RCX / RSEG;
  constexpr bool EVEN = (MX % 2 == 0);
  __shared__ float s_in[MX + RCX];
  __shared__ float2 s_out[NP][RCX];
  __shared__ float2 s_tw[MX];
  const int y = blockIdx.y;
  const int x0 = blockIdx.x * RCX;
  const float* row = f + (size_t)y * W;
  for (int i = threadIdx.x; i < MX + RCX; i += blockDim.x) {
    int xx = x0 - MX + i;
    s_in[i] = (xx >= 0 && xx < W) ? row[xx] : 0.0f;
  }
  for (int i = threadIdx.x; i < MX; i += blockDim.x) s_tw[i] = twx[i];
  __syncthreads();
  const float inv = rsqrtf((float)MX);
  if (threadIdx.x < NP * NSEG) {
    const int p = threadIdx.x / NSEG, s = threadIdx.x % NSEG;
    const int xs = s * RSEG;              // segment start relative to x0
    if (p == 0) {
      // kx = 0 (pole 1) and, for even Mx, kx = Mx/2 (pole -1): real resonators
      float a0 = 0.f, ah = 0.f;
      for (int m = 0; m < MX; ++m) {
        float v = s_in[MX + xs - 1 - m];
        a0 += v;
        ah += (m & 1) ? -v : v;
      }
      for (int i = 0; i < RSEG; ++i) {
        const int xi = xs + i;
        const float comb = s_in[MX + xi] - s_in[xi];
        a0 = a0 + comb;
        ah = -ah + comb;
        s_out[0][xi] = EVEN ? make_float2(a0 * inv, ah * inv) : make_float2(a0 * inv, 0.f);
      }
    } else {
      float2 a = make_float2(0.f, 0.f);
      for (int m = 0; m < MX; ++m) {
        float v = s_in[MX + xs - 1 - m];
        float2 w = s_tw[(p * m) % MX];
        a.x += w.x * v;
        a.y += w.y * v;
      }
      const float2 w1 = s_tw[p];
      for (int i = 0; i < RSEG; ++i) {
        const int xi = xs + i;
        const float comb = s_in[MX + xi] - s_in[xi];
        a = cmul(w1, a);
        a.x += comb;
        s_out[p][xi] = cscale(a, inv);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NP * RCX; i += blockDim.x) {
    const int p = i / RCX, xi = i % RCX;
    if (x0 + xi < W) rs[((size_t)p * H + y) * W + x0 + xi] = s_out[p][xi];
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
};

// (value, index) argmax with the first (lowest-index) maximum winning.
__device__ __forceinline__ void amax_merge(float& v, int& i, float v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

template <int MX, int MY, int MZ>
__global__ void __launch_bounds__(256) k_pixel(PixArgs a) {
  using SH = Shape<MX, MY, MZ>;
  constexpr int NP = SH::NP, NXH = SH::NXH, NCOL = SH::NCOL, NCOLP = SH::NCOLP, PPB = SH::PPB;
  constexpr bool EVEN = SH::EVEN;

  __shared__ float2 s_u[SH::U_ELEMS];            // Hann-z stage, later Q and T
  __shared__ float2 s_b[SH::A_ELEMS];            // Hann-y stage
  __shared__ float s_rv[256];
  __shared__ int s_ri[256];
  __shared__ float2 s_twz[MZ], s_twA[MZ], s_twy[MY];

  const int tid = threadIdx.x;
  const int ps = tid / NCOLP, c = tid % NCOLP;
  const int xblocks = (a.W + PPB - 1) / PPB;
  const int xb = blockIdx.x % xblocks, yb = blockIdx.x / xblocks;
  const int x = xb * PPB + ps;
  const bool px_ok = x < a.W;
  const bool col_ok = px_ok && c < NCOL;
  const int p = c / MY, ky = c % MY;
  const int y0 = yb * a.TY;
  const int y1 = min(a.H, y0 + a.TY);

  for (int i = tid; i < MZ; i += 256) { s_twz[i] = a.twz[i]; s_twA[i] = a.twA[i]; }
  for (int i = tid; i < MY; i += 256) s_twy[i] = a.twy[i];
  __syncthreads();

  float2* s_a = s_u;                                   // [PPB][NCOL][MZ]
  float2* s_q = s_u;                                   // [PPB][NXH][MY]
  float2* s_t = s_u + PPB * NXH * MY;                  // [PPB][NXH][NVY_MAX]
  const int nvx = a.nvx, nvy = a.nvy, nv = a.nv;

  // Column sliding DFT: seed with the direct DFT of the My rows above y0.
  float2 acol = make_float2(0.f, 0.f);
  if (col_ok) {
    for (int m = 0; m < MY; ++m) {
      const int yy = y0 - 1 - m;
      if (yy < 0) break;
      const float2 v = a.rs[((size_t)p * a.H + yy) * a.W + x];
      const float2 w = s_twy[(ky * m) % MY];
      acol = cadd(acol, cmul(w, v));
    }
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
      float2 in = a.rs[((size_t)p * a.H + y) * a.W + x];
      if (y >= MY) in = csub(in, a.rs[((size_t)p * a.H + (y - MY)) * a.W + x]);
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
      const float2* ty = a.tauy + iy * MY;
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
      const float2* tx = a.taux + ix * NXH;
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
    // reduce (value, index) over the pixel's NCOLP threads
#pragma unroll
    for (int off = (NCOLP < 64 ? NCOLP : 64) / 2; off > 0; off >>= 1) {
      const float v2 = __shfl_xor(bv, off, 64);
      const int i2 = __shfl_xor(bi, off, 64);
      amax_merge(bv, bi, v2, i2);
    }
    if (NCOLP > 64) {
      s_rv[tid] = bv;
      s_ri[tid] = bi;
      lds_barrier();
      for (int wv = 1; wv < NCOLP / 64; ++wv) amax_merge(bv, bi, s_rv[(tid ^ (wv * 64))], s_ri[(tid ^ (wv * 64))]);
      lds_barrier();
    }
    const int istar = (bi < nv) ? bi : 0;   // no finite candidate: fall back to index 0

    // ---- background estimate (eq. 4) with the coefficients of the chosen
    // velocity (eq. 8 at the bins; Hermitian weights folded into the table)
    const int hsel = (a.vmode == 2) ? nv : istar;
    float acc = 0.f;
    if (col_ok && p <= a.bx) {
      const int kyc = (2 * ky <= MY) ? ky : ky - MY;
      if (kyc >= -a.by && kyc <= a.by) {
        const float2* h = a.htab + (((size_t)hsel * (a.bx + 1) + p) * (2 * a.by + 1) + (kyc + a.by)) * MZ;
#pragma unroll
        for (int kz = 0; kz < MZ; ++kz) acc += h[kz].x * X[kz].x - h[kz].y * X[kz].y;
      }
    }
#pragma unroll
    for (int off = (NCOLP < 64 ? NCOLP : 64) / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
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
      const float idel = (a.ring_delayed != nullptr && xs >= 0 && ys >= 0) ? a.ring_delayed[(size_t)ys * a.W + xs] : 0.f;
      a.out[pix] = idel - acc;
      if (a.vmode == 2) {
        a.vxy[pix] = make_float2(a.fvx, a.fvy);
        a.vidx[pix] = -1;
      } else {
        a.vxy[pix] = make_float2(a.gx[istar % nvx], a.gy[istar / nvx]);
        a.vidx[pix] = istar;
      }
    }
#pragma unroll
    for (int k = 0; k < MZ; ++k) X[k] = Xn[k];
  }
}

// ---------------------------------------------------------------------------
// Full spectrum S(k; n) = sqrt(Mz) * X at chosen anchors, unpacked to
// [npix][Mx][My][Mz] interleaved complex.
template <int MX, int MY, int MZ>
__global__ void k_spectrum(const float2* __restrict__ st, int W, const int* __restrict__ xy, int npix,
                           float2* __restrict__ out) {
  using SH = Shape<MX, MY, MZ>;
  constexpr int N = MX * MY * MZ;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= npix * N) return;
  const int ip = gid / N, b = gid % N;
  int kx = b / (MY * MZ), kyy = (b / MZ) % MY, kz = b % MZ;
  const size_t pix = (size_t)xy[2 * ip + 1] * W + xy[2 * ip];
  const float2* X = st + pix * SH::NCOL * MZ;
  bool cj = false;
  if (2 * kx > MX) { kx = MX - kx; kyy = (MY - kyy) % MY; kz = (MZ - kz) % MZ; cj = true; }
  float2 r;
  if (kx == 0 || (SH::EVEN && 2 * kx == MX)) {
    const float2 u = X[kyy * MZ + kz];
    if (!SH::EVEN) r = u;
    else {
      const float2 w = X[((MY - kyy) % MY) * MZ + (MZ - kz) % MZ];
      if (kx == 0) r = make_float2(0.5f * (u.x + w.x), 0.5f * (u.y - w.y));
      else         r = make_float2(0.5f * (u.y + w.y), -0.5f * (u.x - w.x));
    }
  } else {
    r = X[(kx * MY + kyy) * MZ + kz];
  }
  if (cj) r = cconj(r);
  out[gid] = cscale(r, sqrtf((float)MZ));
}

// ---------------------------------------------------------------------------
// Launchers
template <int MX, int MY, int MZ>
static hipError_t launch_pixel_t(const PixArgs& a, hipStream_t s) {
  using SH = Shape<MX, MY, MZ>;
  const int xblocks = (a.W + SH::PPB - 1) / SH::PPB;
  const int yblocks = (a.H + a.TY - 1) / a.TY;
  hipLaunchKernelGGL((k_pixel<MX, MY, MZ>), dim3(xblocks * yblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int MX>
static hipError_t launch_row_t(const float* f, float2* rs, const float2* twx, int H, int W, hipStream_t s) {
  dim3 grid((W + RCX - 1) / RCX, H);
  hipLaunchKernelGGL((k_row<MX>), grid, dim3(256), 0, s, f, rs, twx, H, W);
  return hipGetLastError();
}

template <int MX, int MY, int MZ>
static hipError_t launch_spec_t(const float2* st, int W, const int* xy, int npix, float2* out, hipStream_t s) {
  const int n = npix * MX * MY * MZ;
  hipLaunchKernelGGL((k_spectrum<MX, MY, MZ>), dim3((n + 255) / 256), dim3(256), 0, s, st, W, xy, npix, out);
  return hipGetLastError();
}

bool shape_supported(int mx, int my, int mz) {
  return (mx == 8 && my == 8 && mz == 4) || (mx == 16 && my == 16 && mz == 8) || (mx == 9 && my == 9 && mz == 5);
}

int planes_for(int mx) { return (mx % 2 == 0) ? mx / 2 : (mx + 1) / 2; }

hipError_t launch_pixel(int mx, int my, int mz, const PixArgs& a, hipStream_t s) {
  if (mx == 8 && my == 8 && mz == 4) return launch_pixel_t<8, 8, 4>(a, s);
  if (mx == 16 && my == 16 && mz == 8) return launch_pixel_t<16, 16, 8>(a, s);
  if (mx == 9 && my == 9 && mz == 5) return launch_pixel_t<9, 9, 5>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_row(int mx, const float* f, float2* rs, const float2* twx, int H, int W, hipStream_t s) {
  if (mx == 8) return launch_row_t<8>(f, rs, twx, H, W, s);
  if (mx == 16) return launch_row_t<16>(f, rs, twx, H, W, s);
  if (mx == 9) return launch_row_t<9>(f, rs, twx, H, W, s);
  return hipErrorInvalidValue;
}

hipError_t launch_spectrum(int mx, int my, int mz, const float2* st, int W, const int* xy, int npix, float2* out,
                           hipStream_t s) {
  if (mx == 8 && my == 8 && mz == 4) return launch_spec_t<8, 8, 4>(st, W, xy, npix, out, s);
  if (mx == 16 && my == 16 && mz == 8) return launch_spec_t<16, 16, 8>(st, W, xy, npix, out, s);
  if (mx == 9 && my == 9 && mz == 5) return launch_spec_t<9, 9, 5>(st, W, xy, npix, out, s);
  return hipErrorInvalidValue;
}

hipError_t launch_ingest(const float* in, float* slot, long long n, unsigned long long* nonfinite, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_ingest, dim3((unsigned)blocks), dim3(256), 0, s, in, slot, n, nonfinite);
  return hipGetLastError();
}

}  // namespace rmdf
