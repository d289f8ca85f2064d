// rmdf_pixel16.hip - launcher of the 16x16x8 wave-per-anchor pixel kernel
// (the work tile is in rmdf_pixel16.h).
#include <hip/hip_runtime.h>

#include "rmdf_pixel16.h"

namespace rmdf {
namespace p16 {

// Two workgroups (8 wavefronts) per CU: measured as fast as three, and the
// 256-register budget keeps each wavefront's whole row (state, next row's
// prefetched state) in registers.
template <int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_pixel16(PixArgs a) {
  __shared__ __align__(16) char smem[SMEM16];
  const int xblocks = (a.W + WAVES - 1) / WAVES;
  pixel16_tile<MODE>(a, a.ring_delayed, blockIdx.x % xblocks, blockIdx.x / xblocks, smem);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_pixel16_feat(PixArgs a) {
  __shared__ __align__(16) char smem[SMEM16];
  const int xblocks = (a.W + WAVES - 1) / WAVES;
  pixel16_tile<1>(a, a.ring_delayed, blockIdx.x % xblocks, blockIdx.x / xblocks, smem);
}

__global__ void __launch_bounds__(256) k_finish16(PixArgs a, const float* vc, float thr) {
  const long long pix = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pix >= (long long)a.H * a.W) return;
  finish16(a, a.ring_delayed, vc, thr, (int)(pix % a.W), (int)(pix / a.W));
}

}  // namespace p16

bool pixel16_eligible(int mx, int my, int mz, int nvx, int nvy) {
  return mx == 16 && my == 16 && mz == 8 && nvx <= p16::NV1_MAX && nvy <= p16::NV1_MAX;
}

hipError_t launch_pixel16(const PixArgs& a, int mode, hipStream_t s) {
  const int xblocks = (a.W + p16::WAVES - 1) / p16::WAVES;
  const int yblocks = (a.H + a.TY - 1) / a.TY;
  if (mode == 0) hipLaunchKernelGGL(p16::k_pixel16<0>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else if (mode == 1) hipLaunchKernelGGL(p16::k_pixel16_feat, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(p16::k_pixel16<2>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finish16(const PixArgs& a, const float* vc, float thr, hipStream_t s) {
  const long long n = (long long)a.H * a.W;
  hipLaunchKernelGGL(p16::k_finish16, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, a, vc, thr);
  return hipGetLastError();
}

}  // namespace rmdf
