// rmdf_probe.hip - HBM streaming probe: the practical ceiling that the
// per-pixel kernel's achieved bandwidth is compared with.  Not part of the
// filter.  Grid-stride passes of 16-byte accesses over a device buffer:
//   kind 0  read   (each workgroup reduces what it read to one float, so the
//                   loads cannot be dropped; n_blocks floats written)
//   kind 1  write  (a constant)
//   kind 2  copy   (src -> dst)
// nt != 0: non-temporal loads and stores (the form the pixel kernel uses for
// its observer state).
#include <hip/hip_runtime.h>

#include "../../include/rmdf.h"

namespace rmdf {
namespace probe {

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(256) k_read(const v4f* __restrict__ src, size_t n, float* __restrict__ sink) {
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    acc += NT ? __builtin_nontemporal_load(&src[i]) : src[i];
  float s = acc.x + acc.y + acc.z + acc.w;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ float part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

template <bool NT>
__global__ void __launch_bounds__(256) k_write(v4f* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  const v4f v = {1.f, 2.f, 3.f, 4.f};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    if (NT) __builtin_nontemporal_store(v, &dst[i]);
    else dst[i] = v;
  }
}

template <bool NT>
__global__ void __launch_bounds__(256) k_copy(const v4f* __restrict__ src, v4f* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    if (NT) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
    else dst[i] = src[i];
  }
}

}  // namespace probe
}  // namespace rmdf

extern "C" rmdf_status rmdf_hbm_probe(int kind, const void* src, void* dst, size_t bytes, int n_blocks, int nt,
                                      void* stream) {
  using namespace rmdf::probe;
  if (kind < 0 || kind > 2 || n_blocks < 1 || bytes < 16 || (bytes % 16) != 0) return RMDF_E_INVAL;
  if ((kind != 1 && !src) || !dst) return RMDF_E_INVAL;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16) return RMDF_E_INVAL;
  const size_t n = bytes / 16;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const v4f* a = static_cast<const v4f*>(src);
  if (kind == 0) {
    float* sink = static_cast<float*>(dst);
    if (nt) hipLaunchKernelGGL(k_read<true>, dim3(n_blocks), dim3(256), 0, s, a, n, sink);
    else hipLaunchKernelGGL(k_read<false>, dim3(n_blocks), dim3(256), 0, s, a, n, sink);
  } else if (kind == 1) {
    v4f* d = static_cast<v4f*>(dst);
    if (nt) hipLaunchKernelGGL(k_write<true>, dim3(n_blocks), dim3(256), 0, s, d, n);
    else hipLaunchKernelGGL(k_write<false>, dim3(n_blocks), dim3(256), 0, s, d, n);
  } else {
    v4f* d = static_cast<v4f*>(dst);
    if (nt) hipLaunchKernelGGL(k_copy<true>, dim3(n_blocks), dim3(256), 0, s, a, d, n);
    else hipLaunchKernelGGL(k_copy<false>, dim3(n_blocks), dim3(256), 0, s, a, d, n);
  }
  return hipGetLastError() == hipSuccess ? RMDF_OK : RMDF_E_DEVICE;
}
