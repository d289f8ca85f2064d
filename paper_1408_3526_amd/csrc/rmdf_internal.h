// rmdf_internal.h - host-side accessors shared by the single-stream context
// (rmdf_host.hip) and the batched streams (rmdf_batch.hip).  Not part of the
// public ABI.
#pragma once
#include <string>

#include "../../include/rmdf.h"
#include "rmdf_kernels.h"

// Per-pixel kernel arguments of a context (static fields; ring_delayed unset).
rmdf::PixArgs rmdf_internal_pixargs(const rmdf_ctx* c);
const float* rmdf_internal_ring(const rmdf_ctx* c, int* nring, int* dt);
const float2* rmdf_internal_twx(const rmdf_ctx* c);
unsigned long long* rmdf_internal_nonfinite(const rmdf_ctx* c);
void rmdf_internal_shape(const rmdf_ctx* c, int* mx, int* my, int* mz, int* variant);
// Count one frame pushed by someone else (the batched step).
void rmdf_internal_advance(rmdf_ctx* c);
// Mark a context as one stream of a batch (single pushes and state loads are
// then refused: the batch's step advances it).
void rmdf_internal_set_batch_owned(rmdf_ctx* c);
void rmdf_internal_set_create_error(const std::string& m);

namespace rmdf {
// Local spectrum at anchors (xs[i * cstride], ys[i * cstride]) (device arrays);
// launch_spectrum (rmdf_kernels.h) is the interleaved (x, y) form.
hipError_t launch_spectrum_at(int mx, int my, int mz, const float2* st, int W, const int* xs, const int* ys,
                              int cstride, int npix, float2* out, int layout, int newest, hipStream_t s);
// The learned velocity network on n rows of BF16 features (feat[n][1152]):
// vxyc[n][3] = (vx, vy, confidence).  w1p: W1 in operand order (element
// (col, kcol) of the 128 x 1152 matrix at mlp_w1_packed_index(col, kcol));
// w2: BF16 [64][128]; b1, b2, w3 [3][64], b3: FP32.  list != nullptr: rows
// whose confidence is >= thr are appended to list[1..], list[0] counting them
// (the caller zeroes list[0] first).  feat, w1p and w2 16-byte aligned.
hipError_t launch_mlp_infer(const unsigned short* feat, int n, const unsigned short* w1p, const float* b1,
                            const unsigned short* w2, const float* b2, const float* w3, const float* b3, float* vxyc,
                            float thr, int* list, hipStream_t s);
size_t mlp_w1_packed_index(int col, int kcol);
}  // namespace rmdf
