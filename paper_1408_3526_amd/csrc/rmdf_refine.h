// rmdf_refine.h - sub-grid refinement of the velocity peak (velocity mode 3),
// shared by the generic and the wave-per-anchor pixel kernels.
//
// The paper obtains finer velocity resolution by evaluating the
// autocorrelation at finer, non-integer lags (Sec. 2, flow paragraph); mode 3
// additionally interpolates between the grid lags around the first maximum.
#pragma once
#include <hip/hip_runtime.h>

namespace rmdf {

// Sub-grid velocity (velocity mode 3).  The abscissa of the vertex of the
// parabola through (x0, r0), (x1, r1), (x2, r2), x1 when the three values are
// equal: with h0 = x1 - x0, h2 = x2 - x1 and d = r - r1 the parabola is
// r1 + b u + a u^2 (u = x - x1), a h0 h2 (h0 + h2) = d0 h2 + d2 h0 and
// b h0 h2 (h0 + h2) = d2 h0^2 - d0 h2^2; the vertex is at u = -b / (2a).
static __device__ __forceinline__ float peak_vertex(float x0, float r0, float x1, float r1, float x2, float r2) {
  const float h0 = x1 - x0, h2 = x2 - x1, d0 = r0 - r1, d2 = r2 - r1;
  const float den = d0 * h2 + d2 * h0;
  if (den == 0.f) return x1;
  return x1 - 0.5f * (d2 * h0 * h0 - d0 * h2 * h2) / den;
}

// With the first maximum of the smoothed R at best = iy * nvx + ix (value
// rbest), each axis takes the vertex through the peak and its two neighbours
// on that axis; an axis whose peak is on the grid's edge keeps the grid value.
// rv(w) returns the smoothed R at flat index w (where rv exchanges values
// between lanes, best must be the same in all of them).
template <class RV>
static __device__ __forceinline__ float2 refine_peak(const float* gx, const float* gy, int nvx, int nvy, int best,
                                                     float rbest, RV rv) {
  const int ix = best % nvx, iy = best / nvx;
  float vx = gx[ix], vy = gy[iy];
  if (ix > 0 && ix < nvx - 1) vx = peak_vertex(gx[ix - 1], rv(best - 1), vx, rbest, gx[ix + 1], rv(best + 1));
  if (iy > 0 && iy < nvy - 1) vy = peak_vertex(gy[iy - 1], rv(best - nvx), vy, rbest, gy[iy + 1], rv(best + nvx));
  return make_float2(vx, vy);
}

}  // namespace rmdf
