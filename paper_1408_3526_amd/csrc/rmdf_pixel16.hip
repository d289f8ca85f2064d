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
  __shared__ __align__(16) char smem[smem16_bytes<MODE>()];
  const int xblocks = (a.W + WAVES - 1) / WAVES;
  pixel16_tile<MODE>(a, a.ring_delayed, blockIdx.x % xblocks, blockIdx.x / xblocks, smem);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_pixel16_feat(PixArgs a) {
  __shared__ __align__(16) char smem[SMEM16];
  const int xblocks = (a.W + WAVES - 1) / WAVES;
  pixel16_tile<1>(a, a.ring_delayed, blockIdx.x % xblocks, blockIdx.x / xblocks, smem);
}

// Learned mode, second pass.  The network kernel lists the anchors whose
// confidence clears the threshold (list[0] = count, list[1..] = pixel
// indices) after k_conf_reset has zeroed the count; k_finish16 then runs one
// wavefront per listed anchor, its fixed grid striding over the list.
__global__ void k_conf_reset(int* list) {
  if (threadIdx.x == 0) list[0] = 0;
}

constexpr int FINISH_BLOCKS = 2048;

__global__ void __launch_bounds__(256) k_finish16(PixArgs a, const float* vc, float thr, const int* list) {
  const int count = list[0];
  const int nwaves = FINISH_BLOCKS * 4;
  for (int j = blockIdx.x * 4 + (threadIdx.x >> 6); j < count; j += nwaves) {
    const int pix = list[1 + j];
    finish16(a, a.ring_delayed, vc, thr, pix % a.W, pix / a.W);
  }
}

}  // namespace p16

bool pixel16_eligible(int mx, int my, int mz, int nvx, int nvy) {
  return mx == 16 && my == 16 && mz == 8 && nvx <= p16::NV1_MAX && nvy <= p16::NV1_MAX;
}

int p16_block_columns() { return p16::WAVES; }

hipError_t launch_pixel16(const PixArgs& a, int mode, hipStream_t s) {
  const int xblocks = (a.W + p16::WAVES - 1) / p16::WAVES;
  const int yblocks = (a.H + a.TY - 1) / a.TY;
  if (mode == 0) hipLaunchKernelGGL(p16::k_pixel16<0>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else if (mode == 1) hipLaunchKernelGGL(p16::k_pixel16_feat, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else if (mode == 2) hipLaunchKernelGGL(p16::k_pixel16<2>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else if (mode == 3) hipLaunchKernelGGL(p16::k_pixel16<3>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else if (mode == 4) hipLaunchKernelGGL(p16::k_pixel16<4>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else if (mode == 5) hipLaunchKernelGGL(p16::k_pixel16<5>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else if (mode == 6) hipLaunchKernelGGL(p16::k_pixel16<6>, dim3(xblocks * yblocks), dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_conf_reset(int* list, hipStream_t s) {
  hipLaunchKernelGGL(p16::k_conf_reset, dim3(1), dim3(64), 0, s, list);
  return hipGetLastError();
}

hipError_t launch_finish16(const PixArgs& a, const float* vc, float thr, const int* list, hipStream_t s) {
  hipLaunchKernelGGL(p16::k_finish16, dim3(p16::FINISH_BLOCKS), dim3(256), 0, s, a, vc, thr, list);
  return hipGetLastError();
}

}  // namespace rmdf
