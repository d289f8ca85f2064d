// rmdf_kernels.hip - gfx950 kernels of the recursive multidimensional
// prediction-error filter (Kennedy, arXiv:1408.3526).
//
// Per frame (all on one stream):
//   k_row     : row sliding DFT (comb x(n) - x(n-M) into resonators w^k,
//               Sec. 1, eq. 6-7) -> row spectra rs[y][x][plane]; also stores
//               the frame into its delay-ring slot (non-finite samples -> 0,
//               counted)
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

#include "rmdf_device.h"

namespace rmdf {

// ---------------------------------------------------------------------------
// Row sliding DFT.  Block = (row y, chunk of RCX columns).  Each (plane,
// segment) thread seeds its resonators with the direct DFT of the Mx samples
// before the segment, then runs the comb/resonator recursion across RSEG
// columns; results are staged in LDS and written coalesced.
// The single-stream push reads the caller's frame here directly: each block
// also copies its own columns (non-finite samples zeroed and counted) into
// the delay-ring slot, so the frame is read once per push.
template <int MX, bool DIRECT>
__global__ void __launch_bounds__(256) k_row(const float* __restrict__ f, float2* __restrict__ rs,
                                             const float2* __restrict__ twx, int H, int W, float* __restrict__ slot,
                                             unsigned long long* __restrict__ nonfinite) {
  __shared__ __align__(16) char smem[RowShape<MX>::SMEM];
  row_chunk<MX, DIRECT>(f, rs, twx, H, W, blockIdx.y, blockIdx.x * RCX, smem, nonfinite, slot);
}

template <int MX, int MY, int MZ>
__global__ void __launch_bounds__(256) k_pixel(PixArgs a) {
  using SH = Shape<MX, MY, MZ>;
  __shared__ __align__(16) char smem[SH::SMEM];
  const int xblocks = (a.W + SH::PPB - 1) / SH::PPB;
  pixel_tile<MX, MY, MZ>(a, a.ring_delayed, blockIdx.x % xblocks, blockIdx.x / xblocks, smem);
}

// ---------------------------------------------------------------------------
// Full spectrum S(k; n) = sqrt(Mz) * X at chosen anchors, unpacked to
// [npix][Mx][My][Mz] interleaved complex.
// LAYOUT 0: observer state [plane][ky][kz]; 1: the wave-per-anchor 16x16x8
// observer layout [kz / 2][plane][ky] x (kz even, kz odd); 2: ring of 2-D
// spectra [slot][plane][ky] (newest frame in slot newest mod Mz), from which
// X_kz = (1/Mz) sum_m w^(kz m) S2(t - m) is formed here.
template <int MX, int MY, int MZ, int LAYOUT>
__global__ void k_spectrum(const float2* __restrict__ st, int W, const int* __restrict__ xs,
                           const int* __restrict__ ys, int cstride, int npix, float2* __restrict__ out, int newest) {
  using SH = Shape<MX, MY, MZ>;
  constexpr int N = MX * MY * MZ;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= npix * N) return;
  const int ip = gid / N, b = gid % N;
  int kx = b / (MY * MZ), kyy = (b / MZ) % MY, kz = b % MZ;
  const size_t pix = (size_t)ys[(size_t)ip * cstride] * W + xs[(size_t)ip * cstride];
  const float2* S = st + pix * SH::NCOL * MZ;
  auto X = [&](int p, int ky, int k) -> float2 {
    if (LAYOUT == 2) {
      float2 acc = make_float2(0.f, 0.f);
      for (int m = 0; m < MZ; ++m) {
        const int slot = ((newest - m) % MZ + MZ) % MZ;
        float sn, cs;
        sincospif(2.0f * (float)((k * m) % MZ) / MZ, &sn, &cs);
        acc = cadd(acc, cmul(make_float2(cs, sn), S[slot * SH::NCOL + p * MY + ky]));
      }
      return cscale(acc, 1.0f / MZ);
    }
    return S[LAYOUT == 1 ? ((k >> 1) * SH::NCOL + p * MY + ky) * 2 + (k & 1) : (p * MY + ky) * MZ + k];
  };
  bool cj = false;
  if (2 * kx > MX) { kx = MX - kx; kyy = (MY - kyy) % MY; kz = (MZ - kz) % MZ; cj = true; }
  float2 r;
  if (kx == 0 || (SH::EVEN && 2 * kx == MX)) {
    const float2 u = X(0, kyy, kz);
    if (!SH::EVEN) r = u;
    else {
      const float2 w = X(0, (MY - kyy) % MY, (MZ - kz) % MZ);
      if (kx == 0) r = make_float2(0.5f * (u.x + w.x), 0.5f * (u.y - w.y));
      else         r = make_float2(0.5f * (u.y + w.y), -0.5f * (u.x - w.x));
    }
  } else {
    r = X(kx, kyy, kz);
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

template <int MX, bool DIRECT = false>
static hipError_t launch_row_t(const float* f, float2* rs, const float2* twx, int H, int W, float* slot,
                               unsigned long long* nonfinite, hipStream_t s) {
  dim3 grid((W + RCX - 1) / RCX, H);
  hipLaunchKernelGGL((k_row<MX, DIRECT>), grid, dim3(256), 0, s, f, rs, twx, H, W, slot, nonfinite);
  return hipGetLastError();
}

template <int MX, int MY, int MZ, int IL>
static hipError_t launch_spec_t(const float2* st, int W, const int* xs, const int* ys, int cstride, int npix,
                                float2* out, int newest, hipStream_t s) {
  const int n = npix * MX * MY * MZ;
  hipLaunchKernelGGL((k_spectrum<MX, MY, MZ, IL>), dim3((n + 255) / 256), dim3(256), 0, s, st, W, xs, ys, cstride,
                     npix, out, newest);
  return hipGetLastError();
}

bool shape_supported(int mx, int my, int mz) {
  return (mx == 8 && my == 8 && mz == 4) || (mx == 16 && my == 16 && mz == 8) || (mx == 9 && my == 9 && mz == 5);
}

int planes_for(int mx) { return (mx % 2 == 0) ? mx / 2 : (mx + 1) / 2; }

int pixel_block_columns(int mx, int my, int mz) {
  if (mx == 8 && my == 8 && mz == 4) return Shape<8, 8, 4>::PPB;
  if (mx == 16 && my == 16 && mz == 8) return Shape<16, 16, 8>::PPB;
  if (mx == 9 && my == 9 && mz == 5) return Shape<9, 9, 5>::PPB;
  return 1;
}

int auto_tile_rows(int H, int W, int block_columns) {
  // 32 rows per tile where the frame has enough tiles to fill the chip
  // (2048 workgroups, 8 per CU); fewer rows on smaller frames, where a tile's
  // rows run one after another and the launch would otherwise be latency-bound
  const long long xb = (W + block_columns - 1) / block_columns;
  int ty = 32;
  while (ty > 1 && xb * ((H + ty - 1) / ty) < 2048) ty /= 2;
  return ty;
}

hipError_t launch_pixel(int mx, int my, int mz, const PixArgs& a, hipStream_t s) {
  if (mx == 8 && my == 8 && mz == 4) return launch_pixel_t<8, 8, 4>(a, s);
  if (mx == 16 && my == 16 && mz == 8) return launch_pixel_t<16, 16, 8>(a, s);
  if (mx == 9 && my == 9 && mz == 5) return launch_pixel_t<9, 9, 5>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_row(int mx, const float* f, float2* rs, const float2* twx, int H, int W, float* slot,
                      unsigned long long* nonfinite, hipStream_t s, bool direct) {
  if (direct) {
    if (mx == 16) return launch_row_t<16, true>(f, rs, twx, H, W, slot, nonfinite, s);
    return hipErrorInvalidValue;
  }
  if (mx == 8) return launch_row_t<8>(f, rs, twx, H, W, slot, nonfinite, s);
  if (mx == 16) return launch_row_t<16>(f, rs, twx, H, W, slot, nonfinite, s);
  if (mx == 9) return launch_row_t<9>(f, rs, twx, H, W, slot, nonfinite, s);
  return hipErrorInvalidValue;
}

// Anchor i is (xs[i * cstride], ys[i * cstride]) (device arrays).
hipError_t launch_spectrum_at(int mx, int my, int mz, const float2* st, int W, const int* xs, const int* ys,
                              int cstride, int npix, float2* out, int layout, int newest, hipStream_t s) {
  if (npix > (1 << 30) / (mx * my * mz)) return hipErrorInvalidValue;   // thread count must fit an int
  if (mx == 8 && my == 8 && mz == 4) return launch_spec_t<8, 8, 4, 0>(st, W, xs, ys, cstride, npix, out, newest, s);
  if (mx == 16 && my == 16 && mz == 8) {
    if (layout == 2) return launch_spec_t<16, 16, 8, 2>(st, W, xs, ys, cstride, npix, out, newest, s);
    return layout == 1 ? launch_spec_t<16, 16, 8, 1>(st, W, xs, ys, cstride, npix, out, newest, s)
                       : launch_spec_t<16, 16, 8, 0>(st, W, xs, ys, cstride, npix, out, newest, s);
  }
  if (mx == 9 && my == 9 && mz == 5) return launch_spec_t<9, 9, 5, 0>(st, W, xs, ys, cstride, npix, out, newest, s);
  return hipErrorInvalidValue;
}

// Anchors as (x, y) pairs: xy[2 i], xy[2 i + 1].
hipError_t launch_spectrum(int mx, int my, int mz, const float2* st, int W, const int* xy, int npix, float2* out,
                           int layout, int newest, hipStream_t s) {
  return launch_spectrum_at(mx, my, mz, st, W, xy, xy + 1, 2, npix, out, layout, newest, s);
}


}  // namespace rmdf
