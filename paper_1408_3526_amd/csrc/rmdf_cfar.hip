// rmdf_cfar.hip - two-sided cell-averaging CFAR detector on an FP32 image,
// the detection stage after the prediction-error filter (the paper passes
// the filter output to a threshold and a tracker, Sec. 1, without fixing the
// detector).
//
// Per pixel p: training cells = in-frame pixels within Chebyshev distance
// R = guard + train of p but farther than guard; mu and sigma^2 = mean of x
// and of x^2 over them minus mu^2; detection where n > 0 and
// |x(p) - mu| > k sigma.  One workgroup per 64 x 16 output tile: the tile and
// its R-pixel halo are staged in LDS once, box sums along rows (outer and
// guard widths, x and x^2) go to LDS, and each thread sums one output's
// columns.  HBM traffic is one read of the image (plus the halo) and one
// write of the detections; the kernel is a small fraction of a frame.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/rmdf.h"
#include "rmdf_internal.h"

namespace rmdf {
namespace {

constexpr int CF_TW = 64, CF_TH = 16, CF_RMAX = 16;
constexpr int CF_XS = CF_TW + 2 * CF_RMAX;   // staged row stride
constexpr int CF_HR = CF_TH + 2 * CF_RMAX;   // staged rows (at most)

__global__ void __launch_bounds__(256) k_cfar(const float* __restrict__ x, int H, int W, int G, int R, float k,
                                              unsigned char* __restrict__ det, float* __restrict__ level) {
  __shared__ float s_x[CF_HR * CF_XS];
  __shared__ float s_h[4][CF_HR * CF_TW];
  const int tx0 = blockIdx.x * CF_TW, ty0 = blockIdx.y * CF_TH;
  const int hw = CF_TW + 2 * R, hh = CF_TH + 2 * R;
  for (int i = threadIdx.x; i < hh * hw; i += 256) {
    const int r = i / hw, c = i - r * hw;
    const int gy = ty0 - R + r, gx = tx0 - R + c;
    s_x[r * CF_XS + c] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? x[(size_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  // row sums centred on output column c: outer width 2R+1, guard width 2G+1
  for (int i = threadIdx.x; i < hh * CF_TW; i += 256) {
    const int r = i / CF_TW, c = i - r * CF_TW;
    const float* row = s_x + r * CF_XS + c;   // row[R + d] is column c + d
    float so = 0.f, qo = 0.f, si = 0.f, qi = 0.f;
    for (int d = 0; d <= 2 * R; ++d) {
      const float v = row[d];
      so += v;
      qo += v * v;
    }
    for (int d = R - G; d <= R + G; ++d) {
      const float v = row[d];
      si += v;
      qi += v * v;
    }
    s_h[0][i] = so;
    s_h[1][i] = qo;
    s_h[2][i] = si;
    s_h[3][i] = qi;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < CF_TH * CF_TW; i += 256) {
    const int r = i / CF_TW, c = i - r * CF_TW;
    const int gy = ty0 + r, gx = tx0 + c;
    if (gy >= H || gx >= W) continue;
    float so = 0.f, qo = 0.f, si = 0.f, qi = 0.f;
    for (int d = 0; d <= 2 * R; ++d) {
      so += s_h[0][(r + d) * CF_TW + c];
      qo += s_h[1][(r + d) * CF_TW + c];
    }
    for (int d = R - G; d <= R + G; ++d) {
      si += s_h[2][(r + d) * CF_TW + c];
      qi += s_h[3][(r + d) * CF_TW + c];
    }
    // in-frame cells of the outer and guard squares (the frame is a rectangle)
    const int nxo = min(gx + R, W - 1) - max(gx - R, 0) + 1, nyo = min(gy + R, H - 1) - max(gy - R, 0) + 1;
    const int nxi = min(gx + G, W - 1) - max(gx - G, 0) + 1, nyi = min(gy + G, H - 1) - max(gy - G, 0) + 1;
    const int n = nxo * nyo - nxi * nyi;
    float sig = 0.f;
    unsigned char d = 0;
    if (n > 0) {
      const float inv = 1.0f / (float)n;
      const float mu = (so - si) * inv;
      sig = sqrtf(fmaxf((qo - qi) * inv - mu * mu, 0.f));
      d = fabsf(s_x[(r + R) * CF_XS + c + R] - mu) > k * sig ? 1 : 0;
    }
    det[(size_t)gy * W + gx] = d;
    if (level) level[(size_t)gy * W + gx] = sig;
  }
}

}  // namespace
}  // namespace rmdf

extern "C" rmdf_status rmdf_cfar(const float* x_dev, int H, int W, int guard, int train, float k,
                                 unsigned char* det_dev, float* level_dev, void* stream) {
  auto bad = [](const char* m) {
    rmdf_internal_set_create_error(m);
    return RMDF_E_INVAL;
  };
  if (!x_dev || !det_dev) return bad("cfar: NULL image or detection pointer");
  if (H < 1 || W < 1) return bad("cfar: H, W must be >= 1");
  if (guard < 0 || train < 1 || guard + train > rmdf::CF_RMAX) return bad("cfar: need guard >= 0, train >= 1, guard + train <= 16");
  if (!(k >= 0.f) || !(k < INFINITY)) return bad("cfar: k must be finite and >= 0");
  const dim3 grid((W + rmdf::CF_TW - 1) / rmdf::CF_TW, (H + rmdf::CF_TH - 1) / rmdf::CF_TH);
  hipLaunchKernelGGL(rmdf::k_cfar, grid, dim3(256), 0, static_cast<hipStream_t>(stream), x_dev, H, W, guard,
                     guard + train, k, det_dev, level_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    rmdf_internal_set_create_error(std::string("cfar launch: ") + hipGetErrorString(e));
    return RMDF_E_DEVICE;
  }
  return RMDF_OK;
}
