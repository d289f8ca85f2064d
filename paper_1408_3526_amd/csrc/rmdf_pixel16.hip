// rmdf_pixel16.hip - launcher of the 16x16x8 wave-per-anchor pixel kernel
// (the work tile is in rmdf_pixel16.h).
#include <hip/hip_runtime.h>

#include "rmdf_pixel16.h"

namespace rmdf {
namespace p16 {

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_pixel16(PixArgs a) {
  __shared__ __align__(16) char smem[SMEM16];
  const int xblocks = (a.W + WAVES - 1) / WAVES;
  pixel16_tile(a, a.ring_delayed, blockIdx.x % xblocks, blockIdx.x / xblocks, smem);
}

}  // namespace p16

bool pixel16_eligible(int mx, int my, int mz, int nvx, int nvy) {
  return mx == 16 && my == 16 && mz == 8 && nvx <= p16::NV1_MAX && nvy <= p16::NV1_MAX;
}

hipError_t launch_pixel16(const PixArgs& a, hipStream_t s) {
  const int xblocks = (a.W + p16::WAVES - 1) / p16::WAVES;
  const int yblocks = (a.H + a.TY - 1) / a.TY;
  hipLaunchKernelGGL(p16::k_pixel16, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace rmdf
