// rmdf_pixel16.h - per-pixel work tile specialised for the 16x16x8 window.
//
// One wavefront owns one anchor column x and walks down a tile of rows; the
// four wavefronts of a workgroup are independent (wave-level LDS sync only).
// Lane (r, ky) = (lane / 16, lane % 16) holds the (plane, ky) columns
// (r, ky) and (r + 4, ky) of the Hermitian half of the local spectrum
// (plane 0 packs kx = 0 and kx = 8, see rmdf_kernels.hip), i.e. 2 x 8
// complex observer states.  Per row:
//   column sliding DFT        in registers (one resonator per column)
//   deadbeat observer         in registers; state streamed once (8 KB/pixel
//                             read + 8 KB written, prefetched one row ahead)
//   high-pass, Hann along kz  in registers
//   Hann along ky             DPP row rotations (a row of 16 lanes = one plane)
//   unpack of kx = 0 / 8      DPP row mirror (the -ky partner) + register (-kz)
//   Hann along kx, P, stage A LDS exchange of neighbouring planes
//   stage B (ky -> l_y)       lanes = (kx group, l_y); even/odd split in ky
//   stage C (kx -> l_x)       lanes = (l_y group, l_x); smoothing; argmax
//   background estimate       lanes' own columns x coefficient table
// Trigonometric weights of stages B and C are staged in LDS once per tile
// and read into registers for each row's stage.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rmdf_kernels.h"
#include "rmdf_refine.h"
#include "rmdf_wave.h"

namespace rmdf {
namespace p16 {

constexpr int MX = 16, MY = 16, MZ = 8;
constexpr int NXH = 9;            // kx = 0..8
constexpr int NCOL = 128;         // 8 planes x 16 ky
constexpr int WAVES = 4;          // anchors (x) per workgroup
constexpr int SB_PLANES = 9;      // kx = 0 .. 8
constexpr int SB_KZ = 10;         // kz slots per (plane, ky) row: 80 B, so a row of 16
                                  // lanes writing 16 B each covers 64 distinct banks
constexpr int SB_ELEMS = SB_PLANES * MY * SB_KZ;   // float2 per wave
constexpr int NV1_MAX = 21;       // 3 lane groups x 21 <= 64

static __device__ __forceinline__ float2 f2(float x, float y) { return make_float2(x, y); }

// LDS pointers keep their address space so every access is a ds_* instruction
// with an immediate offset (a generic pointer would become a flat access)
#define RMDF_LDS __attribute__((address_space(3)))
#define RMDF_GLOBAL __attribute__((address_space(1)))
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef RMDF_LDS v2f lds_v2;
typedef RMDF_LDS v4f lds_v4;
typedef RMDF_LDS float lds_float;
__device__ __forceinline__ float2 ld2(const lds_v2* p) { const v2f v = *p; return make_float2(v.x, v.y); }
__device__ __forceinline__ float4 ld4(const lds_v2* p) {
  const v4f v = *reinterpret_cast<const lds_v4*>(p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st2(lds_v2* p, float2 v) { *p = v2f{v.x, v.y}; }
// Observer-state traffic is streamed once per frame: non-temporal loads and
// stores (measured 4% faster than cached ones for the whole kernel).
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_stream(float4* p, float a, float b, float c, float d) {
  __builtin_nontemporal_store(v4f{a, b, c, d}, reinterpret_cast<v4f*>(p));
}
__device__ __forceinline__ float2 ld2_stream(const float2* p) {
  const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st2_stream(float2* p, float2 v) {
  __builtin_nontemporal_store(v2f{v.x, v.y}, reinterpret_cast<v2f*>(p));
}
__device__ __forceinline__ void st4(lds_v2* p, float a, float b, float c, float d) {
  *reinterpret_cast<lds_v4*>(p) = v4f{a, b, c, d};
}

template <int CTRL>
static __device__ __forceinline__ float2 dpp2(float2 v) { return f2(dppf<CTRL>(v.x), dppf<CTRL>(v.y)); }

// value held by lane (r, -ky mod 16) of the same row: the row mirrored
// (lane j gets 15 - j), then rotated by one
static __device__ __forceinline__ float2 row_neg(float2 v) { return dpp2<ROR1>(dpp2<MIRROR>(v)); }

static __device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Observer state of the 16x16x8 kernel, per pixel: [kz / 2][plane][ky] x
// (kz even, kz odd) complex, so that one 16-byte load per lane covers 1 KB
// of contiguous memory across the wavefront.  Float2 index of (plane, ky, kz):
static __host__ __device__ __forceinline__ int st16_index(int p, int ky, int kz) {
  return ((kz >> 1) * NCOL + p * MY + ky) * 2 + (kz & 1);
}

// s_b index of (plane kx in [0, 8], ky, kz)
static __device__ __forceinline__ int sb_idx(int kx, int ky, int kz) { return (kx * MY + ky) * SB_KZ + kz; }

// w_8^k X for the eight posterior states (exact rotations for even k)
static __device__ __forceinline__ float2 rot8(float2 a, int k) {
  const float c = 0.70710678118654752f;
  switch (k & 7) {
    case 0: return a;
    case 1: return f2((a.x - a.y) * c, (a.x + a.y) * c);
    case 2: return f2(-a.y, a.x);
    case 3: return f2(-(a.x + a.y) * c, (a.x - a.y) * c);
    case 4: return f2(-a.x, -a.y);
    case 5: return f2((a.y - a.x) * c, -(a.x + a.y) * c);
    case 6: return f2(a.y, -a.x);
    default: return f2((a.x + a.y) * c, (a.y - a.x) * c);
  }
}

// sum_kz P_kz w_8^kz / 512 (stage A of the autocorrelation at l_z = 1: the
// 1/4 per Hann axis and S = sqrt(8) X give P = |h'|^2 * 8 / 4096)
static __device__ __forceinline__ float2 stageA(const float P[MZ]) {
  const float c = 0.70710678118654752f;
  const float re = (P[0] - P[4]) + c * (P[1] - P[3] - P[5] + P[7]);
  const float im = (P[2] - P[6]) + c * (P[1] + P[3] - P[5] - P[7]);
  return f2(re * (1.0f / 512.0f), im * (1.0f / 512.0f));
}

constexpr int LATQ_MAX = 64;      // rows of the lattice coefficient table
constexpr int NC_IT = (NV1_MAX + 2) / 3;   // stage-C iterations per lane
constexpr int ETAB = 8 * 17;        // spatial factors [kx 0..7][ky -8..8], zero outside the band
constexpr size_t SMEM16 = sizeof(float2) * WAVES * SB_ELEMS + sizeof(float4) * 2 * NV1_MAX * 4 +
                          sizeof(float2) * (LATQ_MAX * MZ + ETAB);
// mode 5 (direct column DFT): per wavefront, the row spectra of the last My
// rows ([row mod 16][r] x (plane r, plane r + 4)), and the table w_y^k
constexpr int CRING = MY * 4;             // float4 per wavefront
constexpr size_t SMEM16_DIRECT = SMEM16 + sizeof(float4) * WAVES * CRING + sizeof(float2) * MY;
template <int MODE>
constexpr size_t smem16_bytes() { return MODE == 5 ? SMEM16_DIRECT : SMEM16; }

// Hann along kx, power spectrum and stage A for one (plane kx, ky) column
// of kz values.  The centre comes from registers (CREG) or from LDS; the
// neighbours from LDS.  Plane -1 is the conjugate mirror of plane 1 and
// plane 9 that of plane 7: S(-1, ky, kz) = conj S(1, -ky, -kz),
// S(9, ky, kz) = conj S(7, -ky, -kz).  EDGE: 0 interior, 1 kx = 0, 2 kx = 8.
template <int EDGE, bool CREG>
static __device__ __forceinline__ float2 hann_x_power(const lds_v2* s_b, int ky, int kx, const float2 (&Hc)[MZ],
                                                      float (&P)[MZ]) {
#pragma unroll
  for (int k = 0; k < MZ; k += 2) {
    float4 l, rr, cc;
    if (EDGE == 1) {
      const float2 m0 = ld2(&s_b[sb_idx(1, (MY - ky) & 15, (MZ - k) & 7)]);
      const float2 m1 = ld2(&s_b[sb_idx(1, (MY - ky) & 15, (MZ - k - 1) & 7)]);
      l = make_float4(m0.x, -m0.y, m1.x, -m1.y);
    } else {
      l = ld4(&s_b[sb_idx(kx - 1, ky, k)]);
    }
    if (EDGE == 2) {
      const float2 m0 = ld2(&s_b[sb_idx(7, (MY - ky) & 15, (MZ - k) & 7)]);
      const float2 m1 = ld2(&s_b[sb_idx(7, (MY - ky) & 15, (MZ - k - 1) & 7)]);
      rr = make_float4(m0.x, -m0.y, m1.x, -m1.y);
    } else {
      rr = ld4(&s_b[sb_idx(kx + 1, ky, k)]);
    }
    if (CREG) cc = make_float4(Hc[k].x, Hc[k].y, Hc[k + 1].x, Hc[k + 1].y);
    else cc = ld4(&s_b[sb_idx(kx, ky, k)]);
    const float h0x = 2.f * cc.x - l.x - rr.x, h0y = 2.f * cc.y - l.y - rr.y;
    const float h1x = 2.f * cc.z - l.z - rr.z, h1y = 2.f * cc.w - l.w - rr.w;
    P[k] = h0x * h0x + h0y * h0y;
    P[k + 1] = h1x * h1x + h1y * h1y;
  }
  return stageA(P);
}

// One work tile: 4 adjacent anchor columns starting at 4*xb (one per
// wavefront), rows [yb*TY, yb*TY + TY).  All 256 threads must call it.
// Two floats to BF16 (round to nearest even), packed lo | hi << 16: one
// v_cvt_pk_bf16_f32 on gfx950.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
static __device__ __forceinline__ unsigned int pack_bf16x2(float lo, float hi) {
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned int, v);
}

// cos(m pi / 8) and sin(m pi / 8) for integer m.
__device__ constexpr float cos_pi8(int m) {
  constexpr float t[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                           0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                           -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                           0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
  return t[((m % 16) + 16) % 16];
}
__device__ constexpr float sin_pi8(int m) { return cos_pi8(m - 4); }

// Background estimate of eq. (4) over one lane's plane (kx, ky centred, all
// kz) at a continuous velocity (mode 3).  The coefficient of eq. (8) at the
// bin, times sqrt(Mz) (X = S / sqrt(Mz)), is
//   D_8(kz/8 + phi) / 16 * exp(j pi [ph0 - 7 kz / 8]),
//   phi = (vx kx + vy ky) / 16,  ph0 = -2 (kx m'x + ky m'y) / 16 + 2 phi (m't - 7/2),
// Hermitian weight 2 for kx > 0.  The Dirichlet kernel of order 8 is the mean
// of cos((2i+1) pi w), i = 0..3, i.e. with c = cos(pi w) the Chebyshev sum
//   D_8(w) = c (((16 c^2 - 24) c^2 + 10) c^2 - 1),
// and cos(pi (kz/8 + phi)) comes from one sine/cosine pair of phi.
static __device__ __forceinline__ float pef_plane16(const float2* X, int kx, int kyc, float vx, float vy, int dx,
                                                    int dy, int dt) {
  const float phi = (vx * kx + vy * kyc) * (1.0f / 16.0f);
  float sp, cp;
  sincospif(phi, &sp, &cp);
  const float ph0 = -2.f * (float)(kx * dx + kyc * dy) * (1.0f / 16.0f) + 2.f * phi * ((float)dt - 3.5f);
  float s0, c0;
  sincospif(ph0, &s0, &c0);
  float acc = 0.f;
#pragma unroll
  for (int kz = 0; kz < MZ; ++kz) {
    const float c = cos_pi8(kz) * cp - sin_pi8(kz) * sp;
    const float c2 = c * c;
    const float D = c * (((16.f * c2 - 24.f) * c2 + 10.f) * c2 - 1.f);
    // exp(j pi ph0) exp(-j 7 pi kz / 8)
    const float tc = cos_pi8(7 * kz), ts = -sin_pi8(7 * kz);
    const float er = c0 * tc - s0 * ts, ei = c0 * ts + s0 * tc;
    acc += D * (er * X[kz].x - ei * X[kz].y);
  }
  return acc * ((kx == 0) ? (1.0f / 16.0f) : (2.0f / 16.0f));
}

// F_k = sum_n y_n j^(k n), k = 0..3.
static __device__ __forceinline__ void dft4p(float2 y0, float2 y1, float2 y2, float2 y3, float2* F) {
  const float2 a = f2(y0.x + y2.x, y0.y + y2.y), b = f2(y0.x - y2.x, y0.y - y2.y);
  const float2 c = f2(y1.x + y3.x, y1.y + y3.y), d = f2(y1.x - y3.x, y1.y - y3.y);
  F[0] = f2(a.x + c.x, a.y + c.y);
  F[2] = f2(a.x - c.x, a.y - c.y);
  F[1] = f2(b.x - d.y, b.y + d.x);
  F[3] = f2(b.x + d.y, b.y - d.x);
}

// X_k = (1/8) sum_m x_m exp(+j 2 pi k m / 8): radix-2 decimation in time
// (even and odd samples through dft4p, then the twiddles w^k, w = e^{j pi/4}).
static __device__ __forceinline__ void dft8p_scaled(const float2* x, float2* X) {
  float2 e[4], o[4];
  dft4p(x[0], x[2], x[4], x[6], e);
  dft4p(x[1], x[3], x[5], x[7], o);
  constexpr float h = 0.70710678118654752f;
  const float2 t[4] = {o[0], f2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)), f2(-o[2].y, o[2].x),
                       f2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    X[k] = f2(0.125f * (e[k].x + t[k].x), 0.125f * (e[k].y + t[k].y));
    X[k + 4] = f2(0.125f * (e[k].x - t[k].x), 0.125f * (e[k].y - t[k].y));
  }
}

// MODE: 0 plain search; 1 plain search that also writes the learned model's
// input features; 2 learned mode, first pass: features, and the complete
// fallback result (instantaneous search, i.e. no smoothed-R state, its
// background estimate and output), which finish16 overwrites where the
// network is confident; 3 plain search with the peak refined between grid
// points and the background coefficients evaluated at the refined velocity;
// 4 plain search (or fixed velocity) with the temporal part taken directly
// instead of by the observer: a.st then holds a ring of the last Mz 2-D
// spectra per pixel ([slot][plane][ky], slot = frame mod 8), each frame reads
// the 7 older slots, writes the new one over the oldest, and forms
// X_k = (1/8) sum_m w^(k m) S2(t - m) by an 8-point DFT (the observer's
// posterior in exact arithmetic), halving the state traffic; 5 as 4 with the
// column DFT taken directly as well (sum over the window's My row spectra,
// kept in LDS), with the row pass also direct: no recursion on any axis, the
// non-recursive local spectrum as a comparison point; 6 as 0 for two frames
// per pass (frame pairs): the row's work runs for the pair's first frame
// (row spectra a.rs, output to a.out_first) and then for its second (a.rs2,
// the context's outputs), the second starting from the first's posterior
// and smoothed R held in registers, so that the state and the smoothed R
// are read and written once per pair.
template <int MODE>
static __device__ __forceinline__ void pixel16_tile(const PixArgs& a, const float* ring_delayed, int xb, int yb, char* smem) {
  lds_v2* s_all = (lds_v2*)(smem);
  lds_v4* s_tab = (lds_v4*)(smem + sizeof(float2) * WAVES * SB_ELEMS);  // tabB rows, then tabC rows
  lds_v2* s_g = (lds_v2*)(smem + sizeof(float2) * WAVES * SB_ELEMS + sizeof(float4) * 2 * NV1_MAX * 4);
  const int lane = threadIdx.x & 63;
  // wave-uniform values live in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  lds_v2* s_b = s_all + wv * SB_ELEMS;
  lds_v2* s_q = s_b;                       // [9][16] after Hann along kx
  lds_v2* s_t = s_b + NXH * MY;            // [9][NV1_MAX]
  const int nvx = a.nvx, nvy = a.nvy, nv = a.nv;
  {
    const float4* tb = reinterpret_cast<const float4*>(a.tabB);
    const float4* tc = reinterpret_cast<const float4*>(a.tabC);
    for (int i = threadIdx.x; i < 4 * nvy; i += 256) s_tab[i] = v4f{tb[i].x, tb[i].y, tb[i].z, tb[i].w};
    for (int i = threadIdx.x; i < 4 * nvx; i += 256) s_tab[4 * NV1_MAX + i] = v4f{tc[i].x, tc[i].y, tc[i].z, tc[i].w};
    if (MODE == 5 && threadIdx.x < MY) {
      lds_v2* wy_tab = (lds_v2*)(smem + SMEM16 + sizeof(float4) * WAVES * CRING);
      wy_tab[threadIdx.x] = v2f{a.twy[threadIdx.x].x, a.twy[threadIdx.x].y};
    }
    if (a.gtab != nullptr) {
      for (int i = threadIdx.x; i < a.lat_q * MZ; i += 256) s_g[i] = v2f{a.gtab[i].x, a.gtab[i].y};
      for (int i = threadIdx.x; i < ETAB; i += 256) {
        const int p = i / 17, kc = i % 17 - 8;
        float2 e = f2(0.f, 0.f);
        if (p <= a.bx && kc >= -a.by && kc <= a.by) e = a.etab[p * (2 * a.by + 1) + kc + a.by];
        s_g[LATQ_MAX * MZ + i] = v2f{e.x, e.y};
      }
    }
  }
  __syncthreads();                         // the only workgroup barrier

  const int x = __builtin_amdgcn_readfirstlane(xb * WAVES + wv);
  if (x >= a.W) return;                    // whole wavefront leaves
  const int y0 = yb * a.TY;
  const int y1 = min(a.H, y0 + a.TY);
  if (y0 >= y1) return;

  const int r = lane >> 4, ky = lane & 15;
  const int pA = r, pB = r + 4;
  // stage B lane (g, iy), stage C lane (h, ix)
  const int gB = lane / nvy, iyB = lane % nvy;
  const bool actB = lane < 3 * nvy;
  const int hC = lane / nvx, ixC = lane % nvx;
  const bool actC = lane < 3 * nvx;
  const float2 wy = a.twy[ky];
  const int kyc = (ky <= 8) ? ky : ky - 16;
  // lattice background coefficients (table and spatial factors in LDS)
  const bool lattice = a.gtab != nullptr;

  // row spectra [y][x][plane]: element (row yy) at rsA[yy * rstride]
  const size_t rstride = (size_t)a.W * 8;
  const float2* rsA = a.rs + (size_t)x * 8 + pA;
  const float2* rsB = a.rs + (size_t)x * 8 + pB;

  // column sliding DFT seeded with the 16 rows above the tile (Horner form of
  // the direct DFT: the same resonator run over those rows; rows above the
  // frame are zero).  The 16 loads are issued before the recursion, so a tile
  // start costs one memory latency.
  float2 acA = f2(0.f, 0.f), acB = f2(0.f, 0.f);
  constexpr bool RING = (MODE == 4 || MODE == 5);
  // mode 5: row spectra of the last My rows of this column, slot = row mod 16
  lds_v4* s_cr = (lds_v4*)(smem + SMEM16) + wv * CRING;
  const lds_v2* s_wy = (const lds_v2*)(smem + SMEM16 + sizeof(float4) * WAVES * CRING);
  {
    float2 sA[MY], sB[MY];
#pragma unroll
    for (int i = 0; i < MY; ++i) {
      const int yy = y0 - MY + i;
      sA[i] = (yy >= 0) ? rsA[(size_t)yy * rstride] : f2(0.f, 0.f);
      sB[i] = (yy >= 0) ? rsB[(size_t)yy * rstride] : f2(0.f, 0.f);
    }
    if (MODE == 5) {
      if (ky == 0) {
#pragma unroll
        for (int i = 0; i < MY; ++i) s_cr[((y0 - MY + i) & 15) * 4 + r] = v4f{sA[i].x, sA[i].y, sB[i].x, sB[i].y};
      }
    } else {
#pragma unroll
      for (int i = 0; i < MY; ++i) {
        acA = f2(wy.x * acA.x - wy.y * acA.y + sA[i].x, wy.x * acA.y + wy.y * acA.x + sA[i].y);
        acB = f2(wy.x * acB.x - wy.y * acB.y + sB[i].x, wy.x * acB.y + wy.y * acB.x + sB[i].y);
      }
    }
  }

  // mode 6: the pair's second frame has its own row spectra and column SDFT
  float2 acA2 = f2(0.f, 0.f), acB2 = f2(0.f, 0.f);
  const float2* rsA2 = (MODE == 6) ? a.rs2 + (size_t)x * 8 + pA : rsA;
  const float2* rsB2 = (MODE == 6) ? a.rs2 + (size_t)x * 8 + pB : rsB;
  if (MODE == 6) {
    float2 sA[MY], sB[MY];
#pragma unroll
    for (int i = 0; i < MY; ++i) {
      const int yy = y0 - MY + i;
      sA[i] = (yy >= 0) ? rsA2[(size_t)yy * rstride] : f2(0.f, 0.f);
      sB[i] = (yy >= 0) ? rsB2[(size_t)yy * rstride] : f2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < MY; ++i) {
      acA2 = f2(wy.x * acA2.x - wy.y * acA2.y + sA[i].x, wy.x * acA2.y + wy.y * acA2.x + sA[i].y);
      acB2 = f2(wy.x * acB2.x - wy.y * acB2.y + sB[i].x, wy.x * acB2.y + wy.y * acB2.x + sB[i].y);
    }
  }

  // Rows are software-pipelined: the observer state and row-spectrum samples
  // of row y + 1 are loaded as soon as row y has staged its planes in LDS, so
  // their HBM latency hides behind the flow stages of row y.  State layout:
  // [kz pair][plane][ky] x 2 complex per pixel (st16_index), one 1 KB
  // contiguous run per instruction.
  float4 SnA[MZ / 2], SnB[MZ / 2];
  float2 RA[MZ], RB[MZ];                                 // mode 4: S2(t - m) of the row, m = 0..7
  const int slot0 = __builtin_amdgcn_readfirstlane(a.tcur & 7);   // mode 4: slot of the new frame
  float2 nA, nB, oA = f2(0.f, 0.f), oB = f2(0.f, 0.f);   // rs(y), rs(y - My)
  float2 nA2 = f2(0.f, 0.f), nB2 = f2(0.f, 0.f), oA2 = f2(0.f, 0.f), oB2 = f2(0.f, 0.f);   // mode 6
  {
    if (RING) {
      const float2* src = a.st + ((size_t)y0 * a.W + x) * NCOL * MZ;
#pragma unroll
      for (int m = 1; m < MZ; ++m) {
        const int s = (slot0 - m) & 7;
        RA[m] = ld2_stream(&src[s * NCOL + pA * MY + ky]);
        RB[m] = ld2_stream(&src[s * NCOL + pB * MY + ky]);
      }
    } else {
      const float4* src = reinterpret_cast<const float4*>(a.st + ((size_t)y0 * a.W + x) * NCOL * MZ);
#pragma unroll
      for (int j = 0; j < MZ / 2; ++j) {
        SnA[j] = ld_stream(&src[j * NCOL + pA * MY + ky]);
        SnB[j] = ld_stream(&src[j * NCOL + pB * MY + ky]);
      }
    }
    nA = rsA[(size_t)y0 * rstride];
    nB = rsB[(size_t)y0 * rstride];
    if (MODE != 5 && y0 >= MY) {
      oA = rsA[(size_t)(y0 - MY) * rstride];
      oB = rsB[(size_t)(y0 - MY) * rstride];
    }
    if (MODE == 6) {
      nA2 = rsA2[(size_t)y0 * rstride];
      nB2 = rsB2[(size_t)y0 * rstride];
      if (y0 >= MY) {
        oA2 = rsA2[(size_t)(y0 - MY) * rstride];
        oB2 = rsB2[(size_t)(y0 - MY) * rstride];
      }
    }
  }

  for (int y = y0; y < y1; ++y) {
    const size_t pix = (size_t)y * a.W + x;
    float2 XA[MZ], XB[MZ];
    if (!RING) {
#pragma unroll
      for (int j = 0; j < MZ / 2; ++j) {
        XA[2 * j] = f2(SnA[j].x, SnA[j].y);
        XA[2 * j + 1] = f2(SnA[j].z, SnA[j].w);
        XB[2 * j] = f2(SnB[j].x, SnB[j].y);
        XB[2 * j + 1] = f2(SnB[j].z, SnB[j].w);
      }
    }
    // the row's work for one frame; mode 6 runs it for both frames of a
    // pair: the second frame's observer starts from the first's posterior
    // (still in registers), its smoothing from the first's smoothed R, and
    // the state and smoothed R are stored once, after the second
    float rprev[NC_IT];
    auto frame = [&](auto fc) {
      constexpr int F = decltype(fc)::value;
      constexpr bool LAST = (MODE != 6) || (F == 1);
      float2& cA = F ? acA2 : acA;
      float2& cB = F ? acB2 : acB;
      float2& cnA = F ? nA2 : nA;
      float2& cnB = F ? nB2 : nB;
      float2& coA = F ? oA2 : oA;
      float2& coB = F ? oB2 : oB;
      const float2* frA = F ? rsA2 : rsA;
      const float2* frB = F ? rsB2 : rsB;
      const float* rdel = F ? a.ring_delayed2 : ring_delayed;
      if (MODE == 5) {
        // ---- column DFT, direct: sum_m w_y^(ky m) rs(y - m), m = 0 .. 15
        wave_lds_sync();                   // the previous row's reads of the slot are done
        if (ky == 0) s_cr[(y & 15) * 4 + r] = v4f{cnA.x, cnA.y, cnB.x, cnB.y};
        wave_lds_sync();
        cA = f2(0.f, 0.f);
        cB = f2(0.f, 0.f);
#pragma unroll
        for (int m = 0; m < MY; ++m) {
          const v4f v = s_cr[((y - m) & 15) * 4 + r];
          const float2 w = ld2(&s_wy[(ky * m) & 15]);
          cA = f2(cA.x + w.x * v.x - w.y * v.y, cA.y + w.x * v.y + w.y * v.x);
          cB = f2(cB.x + w.x * v.z - w.y * v.w, cB.y + w.x * v.w + w.y * v.z);
        }
      } else {
        // ---- column sliding DFT
        const float2 iA = f2(cnA.x - coA.x, cnA.y - coA.y), iB = f2(cnB.x - coB.x, cnB.y - coB.y);
        cA = f2(wy.x * cA.x - wy.y * cA.y + iA.x, wy.x * cA.y + wy.y * cA.x + iA.y);
        cB = f2(wy.x * cB.x - wy.y * cB.y + iB.x, wy.x * cB.y + wy.y * cB.x + iB.y);
      }
      if (RING) {
        // ---- temporal DFT over the ring: the new 2-D spectrum (1/sqrt(16)
        // scale) replaces the oldest slot
        RA[0] = f2(0.25f * cA.x, 0.25f * cA.y);
        RB[0] = f2(0.25f * cB.x, 0.25f * cB.y);
        dft8p_scaled(RA, XA);
        dft8p_scaled(RB, XB);
        float2* dst = a.st + pix * NCOL * MZ + slot0 * NCOL;
        st2_stream(&dst[pA * MY + ky], RA[0]);
        st2_stream(&dst[pB * MY + ky], RB[0]);
      } else {
        // ---- deadbeat observer (posterior rotated, innovation shared by all kz)
        float2 sA = f2(0.f, 0.f), sB2 = f2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < MZ; ++k) {
          XA[k] = rot8(XA[k], k);
          XB[k] = rot8(XB[k], k);
          sA = f2(sA.x + XA[k].x, sA.y + XA[k].y);
          sB2 = f2(sB2.x + XB[k].x, sB2.y + XB[k].y);
        }
        // s2 = ac / 4 (1/sqrt(16)); e = (s2 - sum) / 8
        const float2 eA = f2((0.25f * cA.x - sA.x) * 0.125f, (0.25f * cA.y - sA.y) * 0.125f);
        const float2 eB = f2((0.25f * cB.x - sB2.x) * 0.125f, (0.25f * cB.y - sB2.y) * 0.125f);
#pragma unroll
        for (int k = 0; k < MZ; ++k) {
          XA[k] = f2(XA[k].x + eA.x, XA[k].y + eA.y);
          XB[k] = f2(XB[k].x + eB.x, XB[k].y + eB.y);
        }
        float4* dst = reinterpret_cast<float4*>(a.st + pix * NCOL * MZ);
#pragma unroll
        for (int j = 0; j < (LAST ? MZ / 2 : 0); ++j) {
          st_stream(&dst[j * NCOL + pA * MY + ky], XA[2 * j].x, XA[2 * j].y, XA[2 * j + 1].x, XA[2 * j + 1].y);
          st_stream(&dst[j * NCOL + pB * MY + ky], XB[2 * j].x, XB[2 * j].y, XB[2 * j + 1].x, XB[2 * j + 1].y);
        }
      }
      // ---- high-pass + Hann along kz (2X(k) - X(k-1) - X(k+1); the 1/4 per
      // axis is folded into the stage-A weights)
      float2 HA[MZ], HB[MZ];
      {
        float2 V[MZ];
        const bool dc = (lane == 0);       // plane 0 (kx = 0 | kx = 8 packed), ky = 0
#pragma unroll
        for (int k = 0; k < MZ; ++k) {
          const float2 m = XA[(MZ - k) & 7];
          // drop the kx = 0 part: C - (C + conj C(-kz)) / 2
          V[k] = dc ? f2(0.5f * (XA[k].x - m.x), 0.5f * (XA[k].y + m.y)) : XA[k];
        }
#pragma unroll
        for (int k = 0; k < MZ; ++k) {
          const float2 l = V[(k + 7) & 7], rr = V[(k + 1) & 7];
          HA[k] = f2(2.f * V[k].x - l.x - rr.x, 2.f * V[k].y - l.y - rr.y);
          const float2 lb = XB[(k + 7) & 7], rb = XB[(k + 1) & 7];
          HB[k] = f2(2.f * XB[k].x - lb.x - rb.x, 2.f * XB[k].y - lb.y - rb.y);
        }
      }
      // ---- Hann along ky: the neighbours are the adjacent lanes of the row
#pragma unroll
      for (int k = 0; k < MZ; ++k) {
        const float2 dA = dpp2<ROR1>(HA[k]), uA = dpp2<ROR15>(HA[k]);
        HA[k] = f2(2.f * HA[k].x - dA.x - uA.x, 2.f * HA[k].y - dA.y - uA.y);
        const float2 dB = dpp2<ROR1>(HB[k]), uB = dpp2<ROR15>(HB[k]);
        HB[k] = f2(2.f * HB[k].x - dB.x - uB.x, 2.f * HB[k].y - dB.y - uB.y);
      }
      // ---- stage the y,z-windowed planes in LDS, then unpack plane 0:
      // S(0) = (C + conj C(-k)) / 2, S(8) = (C - conj C(-k)) / 2j
      wave_lds_sync();                     // previous row's stage C reads are done
#pragma unroll
      for (int k = 0; k < MZ; k += 2) {
        st4(&s_b[sb_idx(pA, ky, k)], HA[k].x, HA[k].y, HA[k + 1].x, HA[k + 1].y);
        st4(&s_b[sb_idx(pB, ky, k)], HB[k].x, HB[k].y, HB[k + 1].x, HB[k + 1].y);
      }
      wave_lds_sync();
      if (r == 0) {
        // every read of plane 0 precedes every write to it (one wavefront,
        // program order)
        float2 w[MZ];
#pragma unroll
        for (int k = 0; k < MZ; ++k) w[k] = ld2(&s_b[sb_idx(0, (MY - ky) & 15, (MZ - k) & 7)]);
#pragma unroll
        for (int k = 0; k < MZ; k += 2) {
          const float2 u0 = HA[k], u1 = HA[k + 1], w0 = w[k], w1 = w[k + 1];
          st4(&s_b[sb_idx(8, ky, k)], 0.5f * (u0.y + w0.y), -0.5f * (u0.x - w0.x), 0.5f * (u1.y + w1.y),
              -0.5f * (u1.x - w1.x));
          st4(&s_b[sb_idx(0, ky, k)], 0.5f * (u0.x + w0.x), 0.5f * (u0.y - w0.y), 0.5f * (u1.x + w1.x),
              0.5f * (u1.y - w1.y));
        }
      }
      wave_lds_sync();
      // issued here so that their latency overlaps the rest of the flow: this
      // row's smoothed autocorrelation (stage-C lane (hC, ixC) owns the
      // candidates iy = hC + 3j; rows past the grid read the last one) and the
      // delayed input sample
      float idel = 0.f;
      if (MODE != 2 && F == 0) {
        const float* rp = a.rsm + pix * nv;
        const int off0 = hC * nvx + ixC, offl = (nvy - 1) * nvx + ixC;
#pragma unroll
        for (int j = 0; j < NC_IT; ++j) rprev[j] = rp[(unsigned)min(off0 + 3 * j * nvx, offl)];
      }
      {
        const int xs = x - a.dx, ys = y - a.dy;
        if (rdel != nullptr && xs >= 0 && ys >= 0) idel = rdel[(size_t)ys * a.W + xs];
      }
      // next row's state and row-spectrum samples (see the pipeline note);
      // issued after the loads above, which stage C waits for (vector memory
      // completes in order)
      if (y + 1 < y1) {
        if (F > 0) {
        } else if (RING) {
          const float2* src = a.st + (pix + a.W) * NCOL * MZ;
#pragma unroll
          for (int m = 1; m < MZ; ++m) {
            const int s = (slot0 - m) & 7;
            RA[m] = ld2_stream(&src[s * NCOL + pA * MY + ky]);
            RB[m] = ld2_stream(&src[s * NCOL + pB * MY + ky]);
          }
        } else {
          const float4* src = reinterpret_cast<const float4*>(a.st + (pix + a.W) * NCOL * MZ);
#pragma unroll
          for (int j = 0; j < MZ / 2; ++j) {
            SnA[j] = ld_stream(&src[j * NCOL + pA * MY + ky]);
            SnB[j] = ld_stream(&src[j * NCOL + pB * MY + ky]);
          }
        }
        cnA = frA[(size_t)(y + 1) * rstride];
        cnB = frB[(size_t)(y + 1) * rstride];
        if (MODE != 5 && y + 1 >= MY) {
          coA = frA[(size_t)(y + 1 - MY) * rstride];
          coB = frB[(size_t)(y + 1 - MY) * rstride];
        }
      }

      // ---- Hann along kx, power spectrum, stage A: Q(kx, ky) = sum_kz P w_z^kz.
      // Planes -1 and 9 are the conjugate mirrors of planes 1 and 7:
      // S(-1, ky, kz) = conj S(1, -ky, -kz), S(9, ky, kz) = conj S(7, -ky, -kz).
      float2 QA, QB, Q8 = f2(0.f, 0.f);
      float PA[MZ], PB[MZ], P8[MZ];
#pragma unroll
      for (int k = 0; k < MZ; ++k) P8[k] = 0.f;
      if (r == 0) {
        QA = hann_x_power<1, false>(s_b, ky, 0, HA, PA);
        Q8 = hann_x_power<2, false>(s_b, ky, 8, HA, P8);
      } else {
        QA = hann_x_power<0, false>(s_b, ky, pA, HA, PA);
      }
      QB = hann_x_power<0, false>(s_b, ky, pB, HB, PB);
      if (MODE == 1 || MODE == 2) {
        // learned-model input: x = ln(P + eps) - mean over all Mx*My*Mz bins,
        // eps = 1e-6 max P; stored for kx = 0..8 ([kx][ky][kz], BF16); bins
        // with kx = 1..7 stand for their conjugate partner too (weight 2)
        float mx = 0.f;
#pragma unroll
        for (int k = 0; k < MZ; ++k) mx = fmaxf(mx, fmaxf(PA[k], fmaxf(PB[k], r == 0 ? P8[k] : 0.f)));
        mx = group_max<64>(mx);
        const float eps = fmaxf(1e-6f * mx, 1e-30f);
        float sum = 0.f;
#pragma unroll
        for (int k = 0; k < MZ; ++k) {
          PA[k] = __logf(PA[k] + eps);
          PB[k] = __logf(PB[k] + eps);
          P8[k] = (r == 0) ? __logf(P8[k] + eps) : 0.f;
          sum += (r == 0 ? 1.f : 2.f) * PA[k] + 2.f * PB[k] + P8[k];
        }
        sum = group_sum<64>(sum);
        const float mean = sum * (1.0f / (MX * MY * MZ));
        unsigned short* fp = a.feat + pix * (NXH * MY * MZ);
        auto put8 = [&](int kx, const float* L) {
          uint4 u;
          u.x = pack_bf16x2(L[0] - mean, L[1] - mean);
          u.y = pack_bf16x2(L[2] - mean, L[3] - mean);
          u.z = pack_bf16x2(L[4] - mean, L[5] - mean);
          u.w = pack_bf16x2(L[6] - mean, L[7] - mean);
          // streamed: read once, by the network's first layer after the frame
          __builtin_nontemporal_store(v4u{u.x, u.y, u.z, u.w}, reinterpret_cast<v4u*>(fp + (kx * MY + ky) * MZ));
        };
        put8(pA, PA);
        put8(pB, PB);
        if (r == 0) put8(8, P8);
      }
      // even/odd split in ky for stage B: slot 0 = Q(0), slots 1..7 = Q(k)+Q(-k),
      // slot 8 = Q(8), slots 9..15 = Q(16-j) - Q(j-16)... stored by the lane of
      // ky = j as Q(-ky') - Q(ky') with ky' = 16 - j
      const float2 mA = row_neg(QA), mB = row_neg(QB), m8 = row_neg(Q8);
      wave_lds_sync();                     // Hann-x reads of s_b are done (s_q aliases it)
      {
        auto put = [&](int kx, float2 q, float2 m) {
          float2 v;
          if (ky == 0 || ky == 8) v = q;
          else if (ky < 8) v = f2(q.x + m.x, q.y + m.y);
          else v = f2(m.x - q.x, m.y - q.y);
          st2(&s_q[kx * MY + ky], v);
        };
        put(pA, QA, mA);
        put(pB, QB, mB);
        if (r == 0) put(8, Q8, m8);
      }
      wave_lds_sync();

      // ---- stage B: T(kx, l_y) = Q0 + Q8 cos(pi l) + sum_k A_k cos + j B_k sin
      if (actB) {
        float cB[7], sB[7], c8B;
        {
          const lds_float* tb = (const lds_float*)(s_tab) + iyB * 16;
#pragma unroll
          for (int k = 0; k < 7; ++k) { cB[k] = tb[k]; sB[k] = tb[7 + k]; }
          c8B = tb[14];
        }
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
          const int kx = 3 * gB + j;
          const lds_v2* q = s_q + kx * MY;
          float tx = q[0].x + c8B * q[8].x, ty = q[0].y + c8B * q[8].y;
#pragma unroll
          for (int k = 1; k < 8; ++k) {
            const v2f A = q[k], Bv = q[16 - k];
            tx += cB[k - 1] * A.x - sB[k - 1] * Bv.y;
            ty += cB[k - 1] * A.y + sB[k - 1] * Bv.x;
          }
          st2(&s_t[kx * NV1_MAX + iyB], f2(tx, ty));
        }
      }
      wave_lds_sync();

      // ---- stage C: R = T0 + T8 cos(pi l_x) + sum_kx 2 Re[T e^{+j phi}],
      // smoothing and argmax
      float bv = -INFINITY;
      int bi = 0x7fffffff;
      float smv[MODE == 3 ? NC_IT : 1];    // mode 3: this lane's smoothed R, for the peak's neighbours
#pragma unroll
      for (int j = 0; j < (MODE == 3 ? NC_IT : 1); ++j) smv[j] = 0.f;
      if (actC) {
        float cC[7], sC[7], c8C;
        {
          const lds_float* tc = (const lds_float*)(s_tab) + (4 * NV1_MAX + 4 * ixC) * 4;
#pragma unroll
          for (int k = 0; k < 7; ++k) { cC[k] = tc[k]; sC[k] = tc[7 + k]; }
          c8C = tc[14];
        }
#pragma unroll
        for (int j = 0; j < NC_IT; ++j) {
          const int iy = hC + 3 * j;
          if (iy < nvy) {
            float rv = s_t[0 * NV1_MAX + iy].x + c8C * s_t[8 * NV1_MAX + iy].x;
#pragma unroll
            for (int kx = 1; kx < 8; ++kx) {
              const v2f t = s_t[kx * NV1_MAX + iy];
              rv += cC[kx - 1] * t.x - sC[kx - 1] * t.y;
            }
            const int w = iy * nvx + ixC;
            float sm = rv;                   // learned mode: instantaneous R (no smoother state)
            if (MODE != 2) {
              sm = (1.f - a.alpha) * rv + a.alpha * rprev[j];
              if (LAST) a.rsm[pix * nv + w] = sm;
              else rprev[j] = sm;          // the pair's next frame smooths on from here
            }
            if (MODE == 3) smv[j] = sm;
            amax_merge(bv, bi, sm, w);
          }
          __builtin_amdgcn_sched_barrier(0);   // keep one iteration's LDS reads in flight at a time
        }
      }
      group_amax<64>(bv, bi);
      const int istar = (bi < nv) ? bi : 0;
      if (MODE == 2 && lane == 0) a.fidx[pix] = istar;

      // ---- mode 3: the peak refined between grid points; R at (ix, iy) is held
      // by lane (iy mod 3) nvx + ix in its slot iy / 3
      float2 vref = f2(0.f, 0.f);
      if (MODE == 3) {
        const int best = __builtin_amdgcn_readfirstlane(istar);
        auto rv = [&](int w) -> float {
          const int iyn = w / nvx, ixn = w - iyn * nvx;
          const int jn = iyn / 3, src = (iyn - 3 * jn) * nvx + ixn;
          float v = 0.f;
#pragma unroll
          for (int j = 0; j < (MODE == 3 ? NC_IT : 1); ++j)
            if (j == jn) v = smv[j];
          return __shfl(v, src, 64);
        };
        const float rbest = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(bv)));
        vref = refine_peak(a.gx, a.gy, nvx, nvy, best, rbest, rv);
      }

      // ---- background estimate with the chosen velocity's coefficients (the
      // posterior state is still in registers)
      const int hsel = __builtin_amdgcn_readfirstlane((a.vmode == 2) ? nv : istar);
      float acc = 0.f;
      if (MODE == 3) {
        if (kyc >= -a.by && kyc <= a.by) {
          if (pA <= a.bx) acc = pef_plane16(XA, pA, kyc, vref.x, vref.y, a.dx, a.dy, a.dt);
          if (pB <= a.bx) acc += pef_plane16(XB, pB, kyc, vref.x, vref.y, a.dx, a.dy, a.dt);
        }
      } else if (lattice) {
        // coefficient = E(kx, ky) G[(nx kx + ny ky) mod Q][kz]; sum_kz G X first
        const int nq = a.latq[hsel];
        const int nxv = nq >> 16, nyv = (int)(short)(nq & 0xffff);
        const int qm = a.lat_q - 1;
        const lds_v2* gA = s_g + ((nxv * pA + nyv * kyc) & qm) * MZ;
        const lds_v2* gB = s_g + ((nxv * pB + nyv * kyc) & qm) * MZ;
        const lds_v2* e = s_g + LATQ_MAX * MZ + pA * 17 + kyc + 8;   // plane pB = pA + 4
        float2 sA = f2(0.f, 0.f), sB = f2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < MZ; ++k) {
          const v2f g = gA[k], h = gB[k];
          sA.x += g.x * XA[k].x - g.y * XA[k].y;
          sA.y += g.x * XA[k].y + g.y * XA[k].x;
          sB.x += h.x * XB[k].x - h.y * XB[k].y;
          sB.y += h.x * XB[k].y + h.y * XB[k].x;
        }
        const float2 EA = ld2(e), EB = ld2(e + 4 * 17);
        acc = (EA.x * sA.x - EA.y * sA.y) + (EB.x * sB.x - EB.y * sB.y);
      } else if (kyc >= -a.by && kyc <= a.by) {
        const size_t row = (size_t)hsel * (a.bx + 1);
        if (pA <= a.bx) {
          const float2* h = a.htab + ((row + pA) * (2 * a.by + 1) + (kyc + a.by)) * MZ;
#pragma unroll
          for (int k = 0; k < MZ; ++k) acc += h[k].x * XA[k].x - h[k].y * XA[k].y;
        }
        if (pB <= a.bx) {
          const float2* h = a.htab + ((row + pB) * (2 * a.by + 1) + (kyc + a.by)) * MZ;
#pragma unroll
          for (int k = 0; k < MZ; ++k) acc += h[k].x * XB[k].x - h[k].y * XB[k].y;
        }
      }
      acc = group_sum<64>(acc);
      if (lane == 0 && !LAST) {
        if (!isfinite(idel)) idel = 0.f;
        a.out_first[pix] = idel - acc;   // the pair's first frame: its output only
      } else if (lane == 0) {
        if (!isfinite(idel)) idel = 0.f;
        a.out[pix] = idel - acc;
        if (a.vmode == 2) {
          a.vxy[pix] = make_float2(a.fvx, a.fvy);
          a.vidx[pix] = -1;
        } else {
          a.vxy[pix] = (MODE == 3) ? vref : make_float2(a.gx[istar % nvx], a.gy[istar / nvx]);
          a.vidx[pix] = istar;
        }
      }
    };
    frame(std::integral_constant<int, 0>{});
    if constexpr (MODE == 6) frame(std::integral_constant<int, 1>{});
  }
}

// Learned mode, second pass: one wavefront per anchor.  Where the network's
// confidence >= thr: velocity = its (vx, vy), background estimate with eq. (8)
// at that continuous velocity, output.  Elsewhere the wavefront leaves at once
// (the search fallback written by pixel16_tile<2> stands).
static __device__ void finish16(const PixArgs& a, const float* ring_delayed, const float* vc, float thr,
                                int x, int y) {
  const int lane = threadIdx.x & 63;
  const int r = lane >> 4, ky = lane & 15;
  const int pA = r, pB = r + 4;
  const size_t pix = (size_t)y * a.W + x;
  const float conf = vc[3 * pix + 2];
  if (!(conf >= thr)) return;          // the first pass already wrote the search fallback
  const float vx = vc[3 * pix], vy = vc[3 * pix + 1];
  float acc = 0.f;
  const int kyc = (ky <= 8) ? ky : ky - 16;
  if (kyc >= -a.by && kyc <= a.by) {
    const float2* X = a.st + pix * NCOL * MZ;   // layout: st16_index
    for (int h = 0; h < 2; ++h) {
      const int p = h ? pB : pA;
      if (p > a.bx) continue;
      const float2* xc = X + st16_index(p, ky, 0);   // element kz at xc[st16_index(0, 0, kz)]
      float2 xl[MZ];
#pragma unroll
      for (int k = 0; k < MZ; ++k) xl[k] = xc[st16_index(0, 0, k)];
      // eq. (8) at the network's continuous velocity, as in the refined mode
      acc += pef_plane16(xl, p, kyc, vx, vy, a.dx, a.dy, a.dt);
    }
  }
  acc = group_sum<64>(acc);
  if (lane == 0) {
    const int xs = x - a.dx, ys = y - a.dy;
    float idel = (ring_delayed != nullptr && xs >= 0 && ys >= 0) ? ring_delayed[(size_t)ys * a.W + xs] : 0.f;
    if (!isfinite(idel)) idel = 0.f;
    a.out[pix] = idel - acc;
    a.vxy[pix] = make_float2(vx, vy);
    a.vidx[pix] = -2;
  }
}

}  // namespace p16
}  // namespace rmdf
