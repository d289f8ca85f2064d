// rmdf_wave.h - wavefront-level helpers shared by the per-pixel kernels: DPP
// lane exchanges within rows of 16 lanes, lane reads, and reductions over a
// group of 32 or 64 lanes of one wavefront that stay off the LDS permute path
// (a chain of ds_bpermute costs an LDS round trip per level; DPP operands
// come from the neighbouring lanes' registers).
#pragma once
#include <hip/hip_runtime.h>

namespace rmdf {

template <int CTRL>
static __device__ __forceinline__ float dppf(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
static __device__ __forceinline__ int dppi(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
// row_ror:n -> dst[i] = src[(i - n) mod 16] within each row of 16 lanes;
// row_mirror -> dst[i] = src[15 - i]; quad_perm [1,0,3,2] and [2,3,0,1] ->
// dst[i] = src[i ^ 1] and src[i ^ 2]
constexpr int ROR1 = 0x121, ROR4 = 0x124, ROR8 = 0x128, ROR15 = 0x12F, MIRROR = 0x140, QXOR1 = 0xB1,
              QXOR2 = 0x4E;

static __device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// (value, index) argmax with the first (lowest-index) maximum winning: a
// maximum over a total order, so the shape of a reduction built from it does
// not change its result.
static __device__ __forceinline__ void amax_merge(float& v, int& i, float v2, int i2) {
  const bool take = (v2 > v) | ((v2 == v) & (i2 < i));
  v = take ? v2 : v;
  i = take ? i2 : i;
}

// Reductions over groups of G lanes (G = 32: lanes 0-31 and 32-63 are two
// groups; G = 64: the whole wavefront): within each row of 16 lanes by DPP
// (partners lane ^ 1, lane ^ 2, then rotations by 4 and 8, after which every
// lane holds its row's result), then the rows' results read from lanes 0,
// 16, 32 and 48 and combined per group.  The result is the same in every lane
// of a group.  Every lane of the wavefront must be active.
template <int G>
static __device__ __forceinline__ float group_sum(float v) {
  static_assert(G == 32 || G == 64, "groups of 32 or 64 lanes");
  v += dppf<QXOR1>(v);
  v += dppf<QXOR2>(v);
  v += dppf<ROR4>(v);
  v += dppf<ROR8>(v);
  const float r0 = lane_read(v, 0), r1 = lane_read(v, 16), r2 = lane_read(v, 32), r3 = lane_read(v, 48);
  if (G == 64) return (r0 + r1) + (r2 + r3);
  return (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
}

template <int G>
static __device__ __forceinline__ float group_max(float v) {
  static_assert(G == 32 || G == 64, "groups of 32 or 64 lanes");
  v = fmaxf(v, dppf<QXOR1>(v));
  v = fmaxf(v, dppf<QXOR2>(v));
  v = fmaxf(v, dppf<ROR4>(v));
  v = fmaxf(v, dppf<ROR8>(v));
  const float r0 = lane_read(v, 0), r1 = lane_read(v, 16), r2 = lane_read(v, 32), r3 = lane_read(v, 48);
  if (G == 64) return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
  return (threadIdx.x & 32) ? fmaxf(r2, r3) : fmaxf(r0, r1);
}

template <int G>
static __device__ __forceinline__ void group_amax(float& v, int& i) {
  static_assert(G == 32 || G == 64, "groups of 32 or 64 lanes");
  amax_merge(v, i, dppf<QXOR1>(v), dppi<QXOR1>(i));
  amax_merge(v, i, dppf<QXOR2>(v), dppi<QXOR2>(i));
  amax_merge(v, i, dppf<ROR4>(v), dppi<ROR4>(i));
  amax_merge(v, i, dppf<ROR8>(v), dppi<ROR8>(i));
  float va = lane_read(v, 0), vb = lane_read(v, 32);
  int ia = __builtin_amdgcn_readlane(i, 0), ib = __builtin_amdgcn_readlane(i, 32);
  amax_merge(va, ia, lane_read(v, 16), __builtin_amdgcn_readlane(i, 16));
  amax_merge(vb, ib, lane_read(v, 48), __builtin_amdgcn_readlane(i, 48));
  if (G == 64) {
    amax_merge(va, ia, vb, ib);
    v = va;
    i = ia;
  } else {
    const bool hi = (threadIdx.x & 32) != 0;
    v = hi ? vb : va;
    i = hi ? ib : ia;
  }
}

}  // namespace rmdf
