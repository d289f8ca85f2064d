// rmdf_mlp.hip - kernels of the learned velocity surrogate: a small MLP
// (input: the log power spectrum of a pixel's local window; hidden 128 and 64
// with ReLU; output vx, vy and a confidence logit) trained and evaluated with
// BF16 operands on MFMA and FP32 accumulation.
//
//   k_gemm_nt     C[M][N] = act(A[M][K] . B[N][K]^T + bias)   (v_mfma 32x32x16 bf16;
//                 64 or 128 columns per tile)
//   k_transpose   BF16 / FP32 -> BF16 transpose (operands of the weight-gradient GEMMs)
//   k_head        layer 3 (64 -> 3), loss and its gradient, dH2, dW3/db3 partial sums
//   k_infer_head  layer 3 for inference, confidence = sigmoid(logit)
//   k_adam        Adam update of FP32 master weights + BF16 copy
//   k_mlp_infer   the whole network for inference in one kernel (features
//                 streamed into LDS by direct loads, hidden layers kept in LDS,
//                 confident rows compacted into a list)
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <type_traits>
#include <utility>

#include "../../include/rmdf.h"
#include "rmdf_internal.h"

namespace rmdf {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 64;
constexpr int LDSK = BK + 8;   // bf16 per LDS row (144 B): rows 16-byte aligned, banks spread

enum : int { EPI_NONE = 0, EPI_RELU = 1, EPI_RELU_GRAD = 2 };

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// C = epi(A . B^T + bias).  A: M x K (lda), B: N x K (ldb), BF16 row-major,
// K contiguous.  Output FP32 (Cf) and/or BF16 (Cb), row-major ldc.
// EPI_RELU_GRAD multiplies by (aux[m][n] > 0) where aux is BF16 (ldaux).
// Tile BM_ x BN_ (64 or 128 each), four wavefronts in a 2 x 2 arrangement,
// each owning (BM_ / 2) x (BN_ / 2) of C as (BM_ / 64) x (BN_ / 64) MFMA
// 32x32 accumulators.  With BN_ = 128 a layer of 128 outputs reads its input
// rows once; BM_ = 128 halves the re-reads of B (from L2) per row of A.  K
// advances 64 at a time (128 contiguous bytes per row); the next K slice's
// global loads are issued before the current slice's MFMAs.
template <int BM_, int BN_>
__global__ void __launch_bounds__(256) k_gemm_nt(const unsigned short* __restrict__ A, int lda,
                                                 const unsigned short* __restrict__ B, int ldb, int M, int N, int K,
                                                 const float* __restrict__ bias, int epi,
                                                 const unsigned short* __restrict__ aux, int ldaux,
                                                 float* __restrict__ Cf, unsigned short* __restrict__ Cb, int ldc) {
  constexpr int NB = BN_ / 64, MA = BM_ / 64;   // accumulator columns and rows per wavefront
  __shared__ __align__(16) unsigned short sA[BM_ * LDSK];
  __shared__ __align__(16) unsigned short sB[BN_ * LDSK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * BM_, n0 = blockIdx.x * BN_;
  f32x16 acc[MA][NB];
#pragma unroll
  for (int u = 0; u < MA; ++u)
#pragma unroll
    for (int t = 0; t < NB; ++t)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[u][t][i] = 0.f;
  // loader: 8 bf16 (16 B) per piece; piece q -> row q / (BK / 8), k = (q % (BK / 8)) * 8,
  // so each row's BK values (128 B) are read as one contiguous run
  constexpr int KP = BK / 8;                 // pieces per row
  constexpr int LA = BM_ * KP / 256, LB = BN_ * KP / 256;
  // with a single column of tiles every row of A is read exactly once: stream
  // it past the caches (B, read by every tile, stays cached)
  const bool a_once = (gridDim.x == 1);
  auto load = [&](int k0, uint4 (&va)[LA], uint4 (&vb)[LB]) {
#pragma unroll
    for (int t = 0; t < LA; ++t) {
      const int q = tid + 256 * t, r = q / KP, gk = k0 + (q % KP) * 8;
      va[t] = make_uint4(0, 0, 0, 0);
      if (m0 + r < M && gk < K) {
        const uint4* src = reinterpret_cast<const uint4*>(A + (size_t)(m0 + r) * lda + gk);
        if (a_once) {
          const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src));
          va[t] = make_uint4(v.x, v.y, v.z, v.w);
        } else {
          va[t] = *src;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int q = tid + 256 * t, r = q / KP, gk = k0 + (q % KP) * 8;
      vb[t] = make_uint4(0, 0, 0, 0);
      if (n0 + r < N && gk < K) vb[t] = *reinterpret_cast<const uint4*>(B + (size_t)(n0 + r) * ldb + gk);
    }
  };
  uint4 va[LA], vb[LB];
  load(0, va, vb);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();                      // previous slice's MFMA reads of sA/sB are done
#pragma unroll
    for (int t = 0; t < LA; ++t) {
      const int q = tid + 256 * t;
      *reinterpret_cast<uint4*>(&sA[(q / KP) * LDSK + (q % KP) * 8]) = va[t];
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int q = tid + 256 * t;
      *reinterpret_cast<uint4*>(&sB[(q / KP) * LDSK + (q % KP) * 8]) = vb[t];
    }
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK, va, vb);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int r = lane & 31, kq = kk + (lane >> 5) * 8;
      bf16x8 a[MA];
#pragma unroll
      for (int u = 0; u < MA; ++u) a[u] = *reinterpret_cast<const bf16x8*>(&sA[(wm * 32 * MA + 32 * u + r) * LDSK + kq]);
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sB[(wn * 32 * NB + 32 * t + r) * LDSK + kq]);
#pragma unroll
        for (int u = 0; u < MA; ++u) acc[u][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[u], b, acc[u][t], 0, 0, 0);
      }
    }
  }
  // D layout: column = lane % 32; row = (i / 4) * 8 + (lane / 32) * 4 + i % 4
#pragma unroll
  for (int u = 0; u < MA; ++u)
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int col = n0 + wn * 32 * NB + 32 * t + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = m0 + wm * 32 * MA + 32 * u + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
      if (row < M && col < N) {
        float v = acc[u][t][i] + (bias ? bias[col] : 0.f);
        if (epi == EPI_RELU) v = v > 0.f ? v : 0.f;
        else if (epi == EPI_RELU_GRAD) v = (bf16_float(aux[(size_t)row * ldaux + col]) > 0.f) ? v : 0.f;
        if (Cf) Cf[(size_t)row * ldc + col] = v;
        if (Cb) Cb[(size_t)row * ldc + col] = bf16_bits(v);
      }
    }
  }
}

// out[c][r] = in[r][c] (in: R x C, FP32 when inf != nullptr else BF16)
__global__ void __launch_bounds__(256) k_transpose(const unsigned short* __restrict__ inb, const float* __restrict__ inf,
                                                   int R, int C, unsigned short* __restrict__ out) {
  __shared__ unsigned short tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int r = by + j, c = bx + tx;
    unsigned short v = 0;
    if (r < R && c < C) v = inf ? bf16_bits(inf[(size_t)r * C + c]) : inb[(size_t)r * C + c];
    tile[j][tx] = v;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int c = bx + j, r = by + tx;
    if (c < C && r < R) out[(size_t)c * R + r] = tile[tx][j];
  }
}

// Layer 3 + loss + gradient for a batch of n samples.
//   o = W3 h2 + b3 (W3: 3 x 64, FP32), loss = wv * ((o0-lx)^2 + (o1-ly)^2) / n
//        + BCE(o2, t) / n,  t = [max(|o0-lx|, |o1-ly|) <= half_step]
// Writes dH2 (BF16, masked by h2 > 0), accumulates dW3, db3 (FP32, atomics per
// block) and the loss sum.
__global__ void __launch_bounds__(256) k_head(const unsigned short* __restrict__ h2, const float* __restrict__ W3,
                                              const float* __restrict__ b3, const float* __restrict__ lab, int n,
                                              float wv, float half_step, unsigned short* __restrict__ dh2,
                                              float* __restrict__ dW3, float* __restrict__ db3,
                                              float* __restrict__ loss) {
  __shared__ float sW[3 * 64 + 3];
  for (int i = threadIdx.x; i < 3 * 64; i += 256) sW[i] = W3[i];
  if (threadIdx.x < 3) sW[192 + threadIdx.x] = b3[threadIdx.x];
  __syncthreads();
  const int b = blockIdx.x * 256 + threadIdx.x;
  float d[3] = {0.f, 0.f, 0.f};
  float l = 0.f;
  float hv[64];
  if (b < n) {
    const unsigned short* hp = h2 + (size_t)b * 64;
#pragma unroll
    for (int j = 0; j < 64; ++j) hv[j] = bf16_float(hp[j]);
    float o[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      float s = sW[192 + q];
#pragma unroll
      for (int j = 0; j < 64; ++j) s += sW[q * 64 + j] * hv[j];
      o[q] = s;
    }
    const float ex = o[0] - lab[2 * b], ey = o[1] - lab[2 * b + 1];
    const float t = (fmaxf(fabsf(ex), fabsf(ey)) <= half_step) ? 1.f : 0.f;
    const float sp = 1.f / (1.f + expf(-o[2]));
    const float inv = 1.f / (float)n;
    // BCE with logits, stable form: max(o,0) - o t + log(1 + exp(-|o|))
    l = wv * (ex * ex + ey * ey) * inv + (fmaxf(o[2], 0.f) - o[2] * t + log1pf(expf(-fabsf(o[2])))) * inv;
    d[0] = 2.f * wv * ex * inv;
    d[1] = 2.f * wv * ey * inv;
    d[2] = (sp - t) * inv;
    unsigned short* dp = dh2 + (size_t)b * 64;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
      const float g = sW[j] * d[0] + sW[64 + j] * d[1] + sW[128 + j] * d[2];
      dp[j] = bf16_bits(hv[j] > 0.f ? g : 0.f);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 64; ++j) hv[j] = 0.f;
  }
  // dW3[q][j] += sum_b d[q] hv[j]; reduce over the block through LDS
  for (int q = 0; q < 3; ++q) {
    for (int j = 0; j < 64; ++j) {
      float v = d[q] * hv[j];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if ((threadIdx.x & 63) == 0) atomicAdd(&dW3[q * 64 + j], v);
    }
    float v = d[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&db3[q], v);
  }
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

// Column sums (bias gradients): out[j] = sum_r in[r][j] (in BF16 R x C)
__global__ void __launch_bounds__(256) k_colsum(const unsigned short* __restrict__ in, int R, int C,
                                                float* __restrict__ out) {
  const int j = blockIdx.x;
  float s = 0.f;
  for (int r = threadIdx.x; r < R; r += 256) s += bf16_float(in[(size_t)r * C + j]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ float sp[4];
  if ((threadIdx.x & 63) == 0) sp[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = sp[0] + sp[1] + sp[2] + sp[3];
}

// Inference head: (vx, vy, confidence) per sample.
__global__ void __launch_bounds__(256) k_infer_head(const unsigned short* __restrict__ h2, const float* __restrict__ W3,
                                                    const float* __restrict__ b3, int n, float* __restrict__ vxyc) {
  __shared__ float sW[3 * 64 + 3];
  for (int i = threadIdx.x; i < 3 * 64; i += 256) sW[i] = W3[i];
  if (threadIdx.x < 3) sW[192 + threadIdx.x] = b3[threadIdx.x];
  __syncthreads();
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n) return;
  const unsigned short* hp = h2 + (size_t)b * 64;
  float o[3] = {sW[192], sW[193], sW[194]};
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    const float h = bf16_float(hp[j]);
    o[0] += sW[j] * h;
    o[1] += sW[64 + j] * h;
    o[2] += sW[128 + j] * h;
  }
  vxyc[3 * b] = o[0];
  vxyc[3 * b + 1] = o[1];
  vxyc[3 * b + 2] = 1.f / (1.f + expf(-o[2]));
}

// Adam on FP32 master weights; writes the BF16 copy used by the GEMMs.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, unsigned short* __restrict__ pb, int n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = bf16_bits(pi);
}

__global__ void k_to_bf16(const float* __restrict__ in, unsigned short* __restrict__ out, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = bf16_bits(in[i]);
}


// ---- Inference: the whole network in one kernel -----------------------------
// vxyc[m] = head(relu(W2 . relu(W1 . f_m + b1) + b2)) for BF16 feature rows f_m
// (1152 each), with the rounding points and accumulation order of k_gemm_nt
// (layer 1, ReLU, BF16) -> k_gemm_nt (layer 2, ReLU, BF16) -> k_infer_head:
// every MFMA chain runs over K in the same ascending 16-wide steps from zero,
// the bias is added to the finished sum, and the head is the same FP32 fma
// chain over j, so the outputs equal that three-kernel sequence bit for bit.
//
// A workgroup (four wavefronts) takes IBM rows.  Layer 1 streams the rows'
// features through two LDS stages of 64 features per row, filled by direct
// global->LDS loads (no register staging; the next slice is in flight while
// the current one is multiplied); wavefront w owns output columns
// 32w..32w+31 of every row.  Its W1 operands come from the cache (every
// workgroup reads all of W1, so it stays L2-resident) in an operand-ordered
// copy where one wavefront's load is 1 KB contiguous, one slice ahead.  The
// hidden activations then stay in LDS, and no intermediate touches HBM: per
// row the kernel reads its 2304 feature bytes and writes 12 bytes (plus a list
// entry for a confident row).
constexpr int IK1 = 1152, IN1 = 128, IN2 = 64, INSL = IK1 / BK;   // 18 slices of 64
constexpr int IBM = 128;                  // rows per workgroup
constexpr int ISTAGE = IBM * BK;          // BF16 per LDS stage (128 B per row)
constexpr int IMA = IBM / 32;             // layer-1 accumulators per wavefront
constexpr int IDPW = IBM / 32;            // 1 KB direct loads per wavefront per slice

typedef __attribute__((address_space(3))) void lds_void;

template <class F, int... I>
__device__ __forceinline__ void unroll_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// s_waitcnt vmcnt(0) lgkmcnt(0), then the workgroup barrier.  The direct loads
// count in vmcnt; lgkmcnt(0) makes this wavefront's LDS reads of the stage
// about to be refilled complete before any wavefront passes the barrier.  The
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void wait_all_barrier() {
  __builtin_amdgcn_s_waitcnt((7 << 4));   // vmcnt 0, expcnt free, lgkmcnt 0 (gfx9 fields)
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// W1 operand order: 16-byte unit ((s * 4 + k) * 4 + w) * 64 + lane holds
// W1[32 w + lane % 32][64 s + 16 k + 8 (lane / 32) .. + 8].
__host__ __device__ inline size_t w1_packed_index(int col, int kcol) {
  const int w = col >> 5, r = col & 31, s = kcol / BK, k = (kcol % BK) >> 4, hh = (kcol >> 3) & 1, e = kcol & 7;
  return ((((size_t)(s * 4 + k) * 4 + w) * 64) + hh * 32 + r) * 8 + e;
}

__global__ void __launch_bounds__(256) k_mlp_infer(const unsigned short* __restrict__ F, int n,
                                                   const unsigned short* __restrict__ W1p, const float* __restrict__ b1,
                                                   const unsigned short* __restrict__ W2, const float* __restrict__ b2,
                                                   const float* __restrict__ W3, const float* __restrict__ b3,
                                                   float* __restrict__ vxyc, float thr, int* __restrict__ list) {
  // two stages as separate objects, so that the compiler can tell a read of
  // one from a direct load into the other and adds no wait of its own
  __shared__ __align__(16) unsigned short st0[ISTAGE];
  __shared__ __align__(16) unsigned short st1[ISTAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r32 = lane & 31, h = lane >> 5;
  const int m0 = blockIdx.x * IBM;

  // Stage layout: row r's 64 features are 8 chunks of 16 B, chunk c at slot
  // c ^ (r & 7) of the row's 128 B (the MFMA operand reads then spread over
  // all banks).  Direct load q of wavefront w fills rows 8j..8j+7,
  // j = w * IDPW + q, lane l writing slot l & 7 of row 8j + l / 8, so it
  // reads chunk (l & 7) ^ (l / 8): eight lanes cover one 128-byte line.
  // Rows past n re-read row n - 1 (their results are dropped).
  const unsigned short* src[IDPW];
#pragma unroll
  for (int q = 0; q < IDPW; ++q) {
    const int row = 8 * (wv * IDPW + q) + (lane >> 3);
    src[q] = F + (size_t)min(m0 + row, n - 1) * IK1 + ((lane & 7) ^ (lane >> 3)) * 8;
  }
  auto issue = [&](auto slc) {
    constexpr int SL = decltype(slc)::value;
    if constexpr (SL < INSL) {
      unsigned short* dst = (SL & 1) ? st1 : st0;
#pragma unroll
      for (int q = 0; q < IDPW; ++q)   // non-temporal: each feature byte is read once
        __builtin_amdgcn_global_load_lds((const void*)(src[q] + SL * BK), (lds_void*)(dst + (wv * IDPW + q) * 512),
                                         16, 0, 2);
    }
  };
  const unsigned short* w1p = W1p + (size_t)(wv * 64 + lane) * 8;
  bf16x8 bq[2][4];
  auto load_w1 = [&](auto slc) {
    constexpr int SL = decltype(slc)::value;
    if constexpr (SL < INSL) {
#pragma unroll
      for (int k = 0; k < 4; ++k) bq[SL & 1][k] = *reinterpret_cast<const bf16x8*>(w1p + (size_t)(SL * 4 + k) * 2048);
    }
  };
  f32x16 acc[IMA];
#pragma unroll
  for (int u = 0; u < IMA; ++u)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[u][i] = 0.f;

  // layer 1: slice SL is multiplied while slice SL + 1 loads
  issue(std::integral_constant<int, 0>{});
  load_w1(std::integral_constant<int, 0>{});
  unroll_seq([&](auto slc) {
    constexpr int SL = decltype(slc)::value;
    wait_all_barrier();   // slice SL is in LDS (all wavefronts); slice SL - 1's stage is free
    load_w1(std::integral_constant<int, SL + 1>{});
    issue(std::integral_constant<int, SL + 1>{});
    const unsigned short* a = (SL & 1) ? st1 : st0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = 2 * k + h;
#pragma unroll
      for (int u = 0; u < IMA; ++u) {
        const int row = 32 * u + r32;
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + row * 64 + ((c ^ (row & 7)) * 8));
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bq[SL & 1][k], acc[u], 0, 0, 0);
      }
    }
  }, std::make_integer_sequence<int, INSL>{});
  wait_all_barrier();

  // H1 = bf16(relu(acc + b1)) into LDS: 256 B per row, rows 0-15 of each
  // 32-row block in st0 and rows 16-31 in st1 (local row 16u + row % 16),
  // chunk c at slot c ^ (local row % 16).  MFMA result layout: column
  // lane % 32, row (i / 4) * 8 + (lane / 32) * 4 + i % 4.
  {
    const int col = 32 * wv + r32;
    const float bias = b1[col];
#pragma unroll
    for (int u = 0; u < IMA; ++u)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        unsigned short* base = (i < 8) ? st0 : st1;
        const int lr = 16 * u + ((i >> 2) & 1) * 8 + h * 4 + (i & 3);
        float v = acc[u][i] + bias;
        v = v > 0.f ? v : 0.f;
        base[lr * 128 + (((col >> 3) ^ (lr & 15)) * 8) + (col & 7)] = bf16_bits(v);
      }
  }
  wait_all_barrier();

  // layer 2: IBM / 16 units of 32 rows x 32 columns, unit u = w + 4j
  constexpr int NU = IBM / 16, NJ = (NU + 3) / 4;
  f32x16 acc2[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int u = wv + 4 * j, rb = u >> 1, cb = u & 1;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc2[j][i] = 0.f;
    if (u < NU) {
      const unsigned short* hb = ((r32 < 16) ? st0 : st1) + (16 * rb + (r32 & 15)) * 128;
      const unsigned short* w2p = W2 + (size_t)(32 * cb + r32) * IN1 + 8 * h;
      bf16x8 bv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) bv[k] = *reinterpret_cast<const bf16x8*>(w2p + 16 * k);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int c = 2 * k + h;
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(hb + ((c ^ (r32 & 15)) * 8));
        acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[k], acc2[j], 0, 0, 0);
      }
    }
  }
  wait_all_barrier();

  // H2 = bf16(relu(acc2 + b2)) into st0: 128 B per row, chunk c at slot c ^ (row % 8)
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int u = wv + 4 * j, rb = u >> 1, cb = u & 1;
    if (u >= NU) continue;
    const int col = 32 * cb + r32;
    const float bias = b2[col];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 32 * rb + (i >> 2) * 8 + h * 4 + (i & 3);
      float v = acc2[j][i] + bias;
      v = v > 0.f ? v : 0.f;
      st0[row * 64 + (((col >> 3) ^ (row & 7)) * 8) + (col & 7)] = bf16_bits(v);
    }
  }
  wait_all_barrier();

  // head: thread t < IBM takes row m0 + t (the FP32 chain of k_infer_head)
  if (tid < IBM) {
    const int m = m0 + tid;
    bool ok = false;
    if (m < n) {
      float o0 = b3[0], o1 = b3[1], o2 = b3[2];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const uint4 q = *reinterpret_cast<const uint4*>(st0 + tid * 64 + ((c ^ (tid & 7)) * 8));
        const unsigned int wd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int jj = 8 * c + e;
          const float hv = bf16_float((unsigned short)((e & 1) ? (wd[e >> 1] >> 16) : (wd[e >> 1] & 0xffffu)));
          o0 += W3[jj] * hv;
          o1 += W3[64 + jj] * hv;
          o2 += W3[128 + jj] * hv;
        }
      }
      const float conf = 1.f / (1.f + expf(-o2));
      float* o = vxyc + 3 * (size_t)m;
      o[0] = o0;
      o[1] = o1;
      o[2] = conf;
      ok = (list != nullptr) && (conf >= thr);
    }
    // confident rows into list[1..] (list[0] = count), one atomic per wavefront
    const unsigned long long mask = __ballot(ok);
    if (mask) {
      int base = 0;
      if (lane == 0) base = atomicAdd(list, __popcll(mask));
      base = __shfl(base, 0, 64);
      const int before = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
      if (ok) list[1 + base + before] = m;
    }
  }
}

}  // namespace mlp

hipError_t launch_mlp_infer(const unsigned short* feat, int n, const unsigned short* w1p, const float* b1,
                            const unsigned short* w2, const float* b2, const float* w3, const float* b3, float* vxyc,
                            float thr, int* list, hipStream_t s) {
  if (n < 1 || !feat || !w1p || !w2 || !vxyc || ((uintptr_t)feat & 15) || ((uintptr_t)w1p & 15) ||
      ((uintptr_t)w2 & 15))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp::k_mlp_infer, dim3((n + mlp::IBM - 1) / mlp::IBM), dim3(256), 0, s, feat, n, w1p, b1, w2, b2,
                     w3, b3, vxyc, thr, list);
  return hipGetLastError();
}

size_t mlp_w1_packed_index(int col, int kcol) { return mlp::w1_packed_index(col, kcol); }

}  // namespace rmdf

using namespace rmdf::mlp;

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }
static rmdf_status st_of(hipError_t e) { return e == hipSuccess ? RMDF_OK : RMDF_E_DEVICE; }

extern "C" {

rmdf_status rmdf_mlp_gemm_nt(const void* A, int lda, const void* B, int ldb, int M, int N, int K, const float* bias,
                             int epi, const void* aux, int ldaux, float* Cf, void* Cb, int ldc, void* stream) {
  if (!A || !B || M < 1 || N < 1 || K < 1 || (K % 8) || (lda % 8) || (ldb % 8) || (!Cf && !Cb) || epi < 0 || epi > 2 ||
      (epi == EPI_RELU_GRAD && !aux))
    return RMDF_E_INVAL;
  // 128-row tiles where there are rows enough to fill the chip twice over
  const bool tall = (long long)M >= 128LL * 512;
  const unsigned short* a = (const unsigned short*)A;
  const unsigned short* b = (const unsigned short*)B;
  const unsigned short* x = (const unsigned short*)aux;
  unsigned short* cb = (unsigned short*)Cb;
  if (N >= 128 && tall) {
    dim3 grid((N + 127) / 128, (M + 127) / 128);
    hipLaunchKernelGGL((k_gemm_nt<128, 128>), grid, dim3(256), 0, S(stream), a, lda, b, ldb, M, N, K, bias, epi, x,
                       ldaux, Cf, cb, ldc);
  } else if (N >= 128) {
    dim3 grid((N + 127) / 128, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm_nt<64, 128>), grid, dim3(256), 0, S(stream), a, lda, b, ldb, M, N, K, bias, epi, x,
                       ldaux, Cf, cb, ldc);
  } else {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm_nt<64, 64>), grid, dim3(256), 0, S(stream), a, lda, b, ldb, M, N, K, bias, epi, x,
                       ldaux, Cf, cb, ldc);
  }
  return st_of(hipGetLastError());
}

rmdf_status rmdf_mlp_transpose(const void* in_bf16, const float* in_f32, int R, int C, void* out_bf16, void* stream) {
  if ((!in_bf16 && !in_f32) || !out_bf16 || R < 1 || C < 1) return RMDF_E_INVAL;
  dim3 grid((C + 31) / 32, (R + 31) / 32);
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, S(stream), (const unsigned short*)in_bf16, in_f32, R, C,
                     (unsigned short*)out_bf16);
  return st_of(hipGetLastError());
}

rmdf_status rmdf_mlp_head(const void* h2, const float* W3, const float* b3, const float* labels, int n, float wv,
                          float half_step, void* dh2, float* dW3, float* db3, float* loss, void* stream) {
  if (!h2 || !W3 || !b3 || !labels || n < 1 || !dh2 || !dW3 || !db3 || !loss) return RMDF_E_INVAL;
  hipLaunchKernelGGL(k_head, dim3((n + 255) / 256), dim3(256), 0, S(stream), (const unsigned short*)h2, W3, b3, labels,
                     n, wv, half_step, (unsigned short*)dh2, dW3, db3, loss);
  return st_of(hipGetLastError());
}

rmdf_status rmdf_mlp_colsum(const void* in, int R, int C, float* out, void* stream) {
  if (!in || !out || R < 1 || C < 1) return RMDF_E_INVAL;
  hipLaunchKernelGGL(k_colsum, dim3(C), dim3(256), 0, S(stream), (const unsigned short*)in, R, C, out);
  return st_of(hipGetLastError());
}

rmdf_status rmdf_mlp_infer_head(const void* h2, const float* W3, const float* b3, int n, float* vxyc, void* stream) {
  if (!h2 || !W3 || !b3 || n < 1 || !vxyc) return RMDF_E_INVAL;
  hipLaunchKernelGGL(k_infer_head, dim3((n + 255) / 256), dim3(256), 0, S(stream), (const unsigned short*)h2, W3, b3, n,
                     vxyc);
  return st_of(hipGetLastError());
}

rmdf_status rmdf_mlp_adam(float* p, const float* g, float* m, float* v, void* p_bf16, int n, float lr, float b1,
                          float b2, float eps, int step, void* stream) {
  if (!p || !g || !m || !v || n < 1 || step < 1) return RMDF_E_INVAL;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, S(stream), p, g, m, v, (unsigned short*)p_bf16, n, lr,
                     b1, b2, eps, c1, c2);
  return st_of(hipGetLastError());
}

rmdf_status rmdf_mlp_to_bf16(const float* in, void* out, long long n, void* stream) {
  if (!in || !out || n < 1) return RMDF_E_INVAL;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, S(stream), in, (unsigned short*)out, n);
  return st_of(hipGetLastError());
}

}  // extern "C"
