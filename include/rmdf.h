/*
 * rmdf.h - C ABI of the MI355X recursive multidimensional prediction-error
 * filter (Kennedy, arXiv:1408.3526: "Parallel software implementation of
 * recursive multidimensional digital filters for point-target detection in
 * cluttered infrared scenes").
 *
 * The library turns a stream of monochrome frames I(x, y, t) into
 *   - the prediction-error (whitened) output: the frame delayed by m' minus
 *     the velocity-tuned background estimate (Sec. 2, eq. 1 and 4);
 *   - the per-pixel background velocity from the local 3-D autocorrelation
 *     (Sec. 2, eq. 9-10, argmax on the l_z = 1 slice);
 * using a local 3-D spectrum per pixel that is updated recursively every
 * frame (Sec. 1: sliding DFTs along rows and columns, a deadbeat observer in
 * time; eq. 6-7).
 *
 * Conventions
 *   - Every call returns rmdf_status; no C++ exception crosses the ABI.
 *   - Frames and outputs are DEVICE pointers (HIP), FP32, row-major [y][x],
 *     owned by the caller; they must stay valid until the context's stream
 *     has executed the call.  Host-side arrays (candidate grids, weights) are
 *     copied before the call returns.
 *   - All device work is enqueued on the context's HIP stream; calls return
 *     without waiting.  Synchronise that stream before reading results.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Window lengths Kx, Ky, Kt are the analysis-window lengths M (the DFT
 *     sizes), not the paper's half-widths K (the paper uses M = 2K + 1).
 *   - Outputs are indexed by the window anchor: out[y][x] after the push of
 *     frame t is the whitened value of pixel (x - m'_x, y - m'_y) of frame
 *     t - m'_t, computed from the window whose newest corner is (x, y, t).
 *     Samples outside the frame or before the first frame count as zero.
 *   - Non-finite input samples are replaced by 0 and counted.
 */
#ifndef RMDF_H
#define RMDF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmdf_ctx rmdf_ctx;

typedef enum {
  RMDF_OK = 0,
  RMDF_E_INVAL = -1,        /* invalid argument (message in rmdf_last_error) */
  RMDF_E_NOMEM = -2,        /* device allocation failed                      */
  RMDF_E_DEVICE = -3,       /* no HIP device, or a HIP call/launch failed     */
  RMDF_E_STATE = -4,        /* call out of order (e.g. output before a push)  */
  RMDF_E_UNSUPPORTED = -5   /* window shape without a compiled kernel         */
} rmdf_status;

typedef enum {
  RMDF_VEL_SEARCH = 0,      /* argmax of the smoothed autocorrelation (Sec. 2) */
  RMDF_VEL_LEARNED = 1,     /* learned surrogate, search where confidence low  */
  RMDF_VEL_FIXED = 2,       /* one velocity for every pixel (fixed_vx, fixed_vy) */
  RMDF_VEL_REFINED = 3      /* search, then the peak refined between grid points:
                               per axis, the vertex of the parabola through the
                               first maximum of the smoothed R and its two grid
                               neighbours (an edge peak keeps the grid value);
                               eq. (8) is evaluated at that continuous velocity
                               for each anchor.  The grids must be strictly
                               increasing.  rmdf_velocity returns the refined
                               velocity and the grid peak's index.  (The paper
                               gets finer resolution from finer lag grids,
                               Sec. 2; this interpolates between them.)      */
} rmdf_velocity_mode;

typedef struct {
  int Bx, By;               /* filter half-bandwidth B (eq. 2; W = 2B+1 bins).
                               -1: floor(3M/8) (M = 9 gives the paper's B = 3).
                               Valid: 0 <= B <= floor((M-1)/2).               */
  int delay_x, delay_y, delay_t; /* output delay m' (Sec. 3). -1: floor(M/2)
                               (M = 9, 5 give the paper's m' = K).  0 <= m' < M */
  float alpha;              /* pole of the first-order smoother of R (Sec. 2).
                               < 0: exp(-1/10) (Sec. 3).  Valid: [0, 1).       */
  int velocity_mode;        /* rmdf_velocity_mode                              */
  float fixed_vx, fixed_vy; /* velocity used by RMDF_VEL_FIXED                  */
  float conf_threshold;     /* RMDF_VEL_LEARNED: search below this confidence;
                               a finite value in [0, 1] (checked for every
                               mode; default 0.9)                             */
  int tile_rows;            /* rows per work tile of the pixel kernel; 0: auto
                               (32, halved down to 1 while the frame has fewer
                               than 2048 work tiles)                           */
  int kernel_variant;       /* per-pixel kernel: 0 auto, 1 generic (LDS-staged,
                               any compiled shape), 2 one wavefront per anchor
                               (16x16x8, at most 21 candidates per axis)       */
  int write_features;       /* search mode that also writes the learned model's
                               input features each frame (rmdf_features)       */
  int temporal;             /* temporal part of the local spectrum:
                               RMDF_TEMPORAL_OBSERVER (0, default): the deadbeat
                               observer of Sec. 1, its Mz-bin state updated in
                               place; RMDF_TEMPORAL_RING (1): a ring of the
                               last Mz 2-D spectra per pixel and the Mz-point
                               temporal DFT taken directly each frame (the same
                               spectrum; the non-recursive comparison point of
                               Sec. 5 applied to time only);
                               RMDF_TEMPORAL_DIRECT (2): no recursion on any
                               axis, the non-recursive local spectrum of
                               Sec. 5: every row-spectrum bin is the direct
                               Kx-term DFT sum of its window, every 2-D bin the
                               direct Ky-term sum over the window's row spectra,
                               and the temporal part as in the ring (the same
                               spectrum in exact arithmetic).  The ring and the
                               direct form need the 16x16x8 wave-per-anchor
                               kernel and the search or fixed velocity mode;
                               single contexts only.                          */
} rmdf_params;

enum { RMDF_TEMPORAL_OBSERVER = 0, RMDF_TEMPORAL_RING = 1, RMDF_TEMPORAL_DIRECT = 2 };

/* Fill *p with the defaults above (the -1 / negative markers). */
void rmdf_params_default(rmdf_params *p);

/* Create a filter for H x W frames with window lengths Kx x Ky x Kt and the
 * candidate velocity grid vgrid_x[nvx] x vgrid_y[nvy] (host arrays, pixels per
 * frame; candidate index i = iy * nvx + ix).  p == NULL: defaults.
 * hip_stream: the hipStream_t every call of this context enqueues on; NULL
 * means the device's default (null) stream.
 * Allocates all device state (observer state H*W*Kx*Ky*Kt/2 complex FP32, or
 * the ring of Kt 2-D spectra of the same size with RMDF_TEMPORAL_RING or
 * RMDF_TEMPORAL_DIRECT,
 * smoothed autocorrelation H*W*nvx*nvy FP32, row spectra, a (m'_t+2)-frame
 * delay ring, tables) and zeroes it.
 * Compiled window shapes: 8x8x4, 16x16x8, 9x9x5 (others: RMDF_E_UNSUPPORTED).
 * Errors: RMDF_E_INVAL (H, W < 1 or H > 65535; bad B, m', alpha, conf_threshold; nvx, nvy outside [1, 33],
 * non-finite grid; unknown velocity or temporal mode; RMDF_VEL_REFINED with a
 * grid that is not strictly increasing; out == NULL), RMDF_E_UNSUPPORTED (a
 * mode the chosen kernel lacks: the learned model, write_features and the
 * temporal ring need the 16x16x8 wave-per-anchor kernel; the ring and
 * write_features exclude the learned and refined modes), RMDF_E_DEVICE,
 * RMDF_E_NOMEM. */
rmdf_status rmdf_create(int H, int W, int Kx, int Ky, int Kt,
                        const float *vgrid_x, int nvx, const float *vgrid_y, int nvy,
                        const rmdf_params *p, void *hip_stream, rmdf_ctx **out);

/* Push the next frame (device pointer, H*W FP32) and run the whole per-frame
 * path on the context stream: the row sliding DFT (which also stores the frame
 * into the delay ring), then the per-pixel kernel (column sliding DFT, observer update,
 * high-pass + Hann + power spectrum, autocorrelation on the grid, smoothing,
 * argmax, velocity-tuned background estimate, output).
 * Paper: the frame stream I(n) of Sec. 2 (eq. 1); the local spectrum of eq. (6)
 * updated recursively (Sec. 1: sliding DFTs in x and y, the deadbeat observer
 * in t); the flow estimate of eq. (9)-(10) with its first-order smoother
 * (Sec. 2, flow paragraph); the background estimate of eq. (4) with the
 * coefficients of eq. (8).
 * The frame is read during the call's kernels only (the caller keeps
 * ownership).  Every argument and state check comes before the first launch,
 * so a refused push changes nothing: not the frame count, the delay ring nor
 * the non-finite counter.  Frames smaller than the window are accepted (the
 * samples outside the frame count as zero).
 * Errors: RMDF_E_INVAL (NULL), RMDF_E_STATE (learned mode without weights,
 * or a stream owned by a batch: those advance with rmdf_batch_push),
 * RMDF_E_DEVICE (launch failure). */
rmdf_status rmdf_push_frame(rmdf_ctx *ctx, const float *frame_dev);

/* Push n frames in order (frames_dev: n device pointers, each H*W FP32,
 * read during the call's kernels).  Where the context allows it (16x16x8
 * window on the one-wavefront-per-anchor kernel, the observer form, velocity
 * search or fixed) the frames go through the per-pixel kernel two at a time:
 * one pass over the observer state and the smoothed R serves both (Sec. 1's
 * recursion and Sec. 2's smoother advanced twice per pass), so their HBM
 * traffic per frame halves, at the price of one frame of latency.  The
 * results are those of n rmdf_push_frame calls, bit for bit.  out_dev: NULL,
 * or n device pointers (each may be NULL) that receive each frame's output
 * (H*W FP32, as rmdf_output); rmdf_output and rmdf_velocity then refer to the
 * last frame.  Every argument and state check precedes the first launch.
 * Errors: RMDF_E_INVAL (NULL ctx or frame, n < 1), RMDF_E_STATE (learned mode
 * without weights, or a stream owned by a batch), RMDF_E_DEVICE. */
rmdf_status rmdf_push_frames(rmdf_ctx *ctx, int n, const float *const *frames_dev, float *const *out_dev);

/* Copy the velocity field of the latest frame into caller buffers:
 * vxy_dev[H*W*2] = (vx, vy) per anchor; idx_dev[H*W] = candidate index
 * (-1 where a fixed velocity was used); either may be NULL.
 * Paper: v = l / l_z at the maximum of the smoothed autocorrelation on the
 * l_z = 1 slice (Sec. 2, flow paragraph and eq. 10); the per-pixel velocity
 * the detector hands on (Sec. 1).  Device-to-device copies on the context
 * stream; the buffers are the caller's.
 * Errors: RMDF_E_INVAL (NULL ctx), RMDF_E_STATE before the first push. */
rmdf_status rmdf_velocity(rmdf_ctx *ctx, float *vxy_dev, int *idx_dev);

/* Copy the prediction-error output of the latest frame into out_dev[H*W].
 * Paper: the whitened output I(n - m') - I^(n - m') (Sec. 2, eq. 1 and 4),
 * i.e. the foreground plus noise, delayed by m' (Sec. 3: two frames for the
 * paper's window).  A device-to-device copy on the context stream into the
 * caller's buffer.
 * Errors: RMDF_E_INVAL (NULL), RMDF_E_STATE before the first push. */
rmdf_status rmdf_output(rmdf_ctx *ctx, float *out_dev);

/* Frames pushed so far, and non-finite input samples replaced by zero (the
 * count is read back from the device and synchronises the stream). */
rmdf_status rmdf_frames_pushed(const rmdf_ctx *ctx, long long *n);
rmdf_status rmdf_nonfinite_count(rmdf_ctx *ctx, long long *n);

/* Local 3-D spectrum S(k; n) (eq. 6, newest sample at m = 0) of the latest
 * frame at anchors (xs[i], ys[i]), i < npix (host arrays), written to the
 * device buffer spec_dev[npix][Kx][Ky][Kt] as interleaved complex FP32.
 * Intended for verification.  Errors: RMDF_E_INVAL, RMDF_E_STATE. */
rmdf_status rmdf_spectrum(rmdf_ctx *ctx, int npix, const int *xs, const int *ys, float *spec_dev);

/* Allocation-free form of rmdf_spectrum, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result and errors as
 * rmdf_spectrum, and the same kernel; the anchor coordinates are staged in a
 * fixed device array of the library (RMDF_SPECTRUM_NOALLOC_MAX anchors, 512 KB
 * per GPU, held until the process ends) instead of a buffer the context
 * allocates, and the call makes no hipMalloc/hipFree.  npix above
 * RMDF_SPECTRUM_NOALLOC_MAX: RMDF_E_INVAL.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other host threads, or contexts
 * on other streams) race; calls from one thread do not, since the call
 * returns only after its stream has finished the copy and the kernel. */
enum { RMDF_SPECTRUM_NOALLOC_MAX = 65536 };
rmdf_status rmdf_spectrum_noalloc(rmdf_ctx *ctx, int npix, const int *xs, const int *ys, float *spec_dev);

/* Smoothed autocorrelation R' of the latest frame on the candidate grid,
 * rs_dev[H*W][nvx*nvy] (device, FP32). Errors: RMDF_E_STATE. */
rmdf_status rmdf_smoothed_r(rmdf_ctx *ctx, float *rs_dev);

/* Per-kernel timing with HIP events on the context stream (off by default).
 * which: 0 = pixel kernel, 1 = row sliding-DFT kernel (which also copies the
 * frame into the delay ring), 2 = unused (no separate ingest kernel),
 * 3 = learned-model network (the confident-anchor count reset and the
 * network kernel), 4 = learned-mode finish kernel.
 * rmdf_set_timing: mask bit w times kernel w; 0 = off, -1 = all (each timed
 * launch adds two event records to the stream, so time only what is needed).
 * rmdf_kernel_time returns the summed milliseconds and the number of timed
 * launches since the last reset (reading synchronises the stream). */
rmdf_status rmdf_set_timing(rmdf_ctx *ctx, int mask);
rmdf_status rmdf_kernel_time(rmdf_ctx *ctx, int which, double *ms, long long *launches);

/* ---- Learned velocity surrogate (16x16x8 window) ----------------------
 * Not in the paper: a small network maps each anchor's local power spectrum
 * (the P of eq. 9) to (vx, vy, confidence); where the confidence is below
 * conf_threshold the anchor falls back to the search over the grid (eq. 10
 * without the smoother, which this mode does not keep).  Input features:
 * x = ln(P + 1e-6 max P) minus its mean over all Mx*My*Mz bins, stored for
 * kx = 0..8 as [kx][ky][kz] (1152 BF16 per anchor; P is even, so the other
 * half repeats them and the first layer is kept folded over +-k).
 * Layers: 1152 -> 128 (ReLU) -> 64 (ReLU) -> 3, BF16 weights on MFMA with
 * FP32 accumulation for the first two, FP32 for the last.
 * Weight blob (host, FP32, row-major [out][in]): W1 128x1152, b1 128,
 * W2 64x128, b2 64, W3 3x64, b3 3 (bytes = 4 * 156,035).  The velocity index
 * of an anchor that used the network is -2.  The upload is enqueued on the
 * context stream (after the pushes already queued there, which keep the
 * previous weights) and the call returns once it has completed.
 * Errors: RMDF_E_INVAL (NULL, wrong size, non-finite weight), RMDF_E_STATE
 * (context not in learned mode), RMDF_E_DEVICE. */
rmdf_status rmdf_mlp_set_weights(rmdf_ctx *ctx, const float *blob, size_t bytes);
/* Features of the latest frame, feat_dev[H*W][1152] BF16 (learned mode or
 * write_features).  Errors: RMDF_E_STATE. */
rmdf_status rmdf_features(rmdf_ctx *ctx, void *feat_dev);
/* Network output of the latest frame, vc_dev[H*W][3] = (vx, vy, confidence). */
rmdf_status rmdf_learned_output(rmdf_ctx *ctx, float *vc_dev);
/* The context's network alone on n rows of caller features (feat_dev[n][1152]
 * BF16, device, 16-byte aligned), with the kernel a learned-mode push uses
 * (the whole network in one launch; its outputs equal those of
 * rmdf_mlp_gemm_nt for each hidden layer, ReLU and BF16 output, followed by
 * rmdf_mlp_infer_head, bit for bit): vc_dev[n][3] = (vx, vy, confidence),
 * enqueued on the context stream.  For verification.  Errors: RMDF_E_INVAL
 * (NULL, n < 1, misaligned features), RMDF_E_STATE (not in learned mode, or
 * no weights), RMDF_E_DEVICE. */
rmdf_status rmdf_learned_network(rmdf_ctx *ctx, const void *feat_dev, int n, float *vc_dev);

/* Kernels of the learned model, for training (all asynchronous on `stream`,
 * device pointers; BF16 as uint16).  rmdf_mlp_gemm_nt:
 * C[M][N] = epi(A[M][K] . B[N][K]^T + bias[N]) with A, B BF16 row-major
 * (K contiguous, K, lda, ldb multiples of 8); epi 0 none, 1 ReLU, 2 multiply
 * by (aux[m][n] > 0) (ReLU gradient, aux BF16); output FP32 (Cf) and/or BF16
 * (Cb) with leading dimension ldc.  Errors: RMDF_E_INVAL, RMDF_E_DEVICE. */
rmdf_status rmdf_mlp_gemm_nt(const void *A, int lda, const void *B, int ldb, int M, int N, int K, const float *bias,
                             int epi, const void *aux, int ldaux, float *Cf, void *Cb, int ldc, void *stream);
/* out[c][r] = in[r][c]; input BF16 (in_bf16) or FP32 (in_f32, rounded). */
rmdf_status rmdf_mlp_transpose(const void *in_bf16, const float *in_f32, int R, int C, void *out_bf16, void *stream);
/* Last layer, loss and its gradient for n samples: o = W3 h2 + b3;
 * loss = sum_b [wv ((o0-lx)^2 + (o1-ly)^2) + BCE(o2, t)] / n with
 * t = [max(|o0-lx|, |o1-ly|) <= half_step]; writes dh2 (BF16, masked by
 * h2 > 0); adds into dW3 (3x64), db3 (3) and *loss. */
rmdf_status rmdf_mlp_head(const void *h2, const float *W3, const float *b3, const float *labels, int n, float wv,
                          float half_step, void *dh2, float *dW3, float *db3, float *loss, void *stream);
/* out[j] = sum_r in[r][j], in BF16 R x C (bias gradients). */
rmdf_status rmdf_mlp_colsum(const void *in, int R, int C, float *out, void *stream);
/* Inference head: vxyc[b] = (o0, o1, sigmoid(o2)). */
rmdf_status rmdf_mlp_infer_head(const void *h2, const float *W3, const float *b3, int n, float *vxyc, void *stream);
/* Adam step (FP32 master weights p, gradient g, moments m, v); writes the
 * BF16 copy p_bf16 when non-NULL.  step counts from 1. */
rmdf_status rmdf_mlp_adam(float *p, const float *g, float *m, float *v, void *p_bf16, int n, float lr, float b1,
                          float b2, float eps, int step, void *stream);
rmdf_status rmdf_mlp_to_bf16(const float *in, void *out_bf16, long long n, void *stream);

/* Per-pixel kernel variant the context launches (1 generic, 2 one wavefront
 * per anchor), after resolving kernel_variant = 0. */
rmdf_status rmdf_kernel_variant(const rmdf_ctx *ctx, int *variant);

/* Rows per work tile of the pixel kernel, after resolving tile_rows = 0. */
rmdf_status rmdf_tile_rows(const rmdf_ctx *ctx, int *tile_rows);

/* How the wavefront-per-anchor kernel stores the background coefficients of
 * eq. (8): *lattice_q = 16 s when every candidate velocity (and the fixed
 * velocity in RMDF_VEL_FIXED mode) is a whole multiple of 1/s px/frame for
 * s in {1, 2, 4}; the coefficients then factor into a spatial phase per
 * (kx, ky) and a 16 s x Kt table of the temporal part, held in LDS.
 * *lattice_q = 0: a per-candidate table in device memory is read instead
 * (any other grid, or the generic kernel), or, in RMDF_VEL_REFINED mode, the
 * coefficients are evaluated per anchor at the refined velocity. */
rmdf_status rmdf_coeff_lattice(const rmdf_ctx *ctx, int *lattice_q);

/* Detection stage after the filter (the paper hands the prediction error to a
 * threshold and a tracker, Sec. 1, without fixing the detector): two-sided
 * cell-averaging CFAR on an H x W FP32 device image x_dev (row-major, e.g.
 * what rmdf_output wrote).  Per pixel, the training cells are the in-frame
 * pixels within Chebyshev distance guard + train that lie outside the guard
 * square (which holds the pixel itself); mu = their mean, sigma^2 = the mean
 * of their squares minus mu^2 (FP32), and det_dev[p] = 1 where there is at
 * least one training cell and |x - mu| > k sigma, else 0 (H*W bytes, device).
 * level_dev: H*W sigma values (device), or NULL.  guard >= 0, train >= 1,
 * guard + train <= 16, k finite and >= 0; otherwise RMDF_E_INVAL with the
 * message in rmdf_last_error(NULL).  Buffers are the caller's; the call is
 * enqueued on `stream` (NULL: the default stream) and allocates nothing. */
rmdf_status rmdf_cfar(const float *x_dev, int H, int W, int guard, int train, float k,
                      unsigned char *det_dev, float *level_dev, void *stream);

/* HBM streaming probe (measurement utility, not part of the filter): one
 * grid-stride pass of 16-byte accesses over `bytes` of device memory on
 * `stream` (NULL: default stream), n_blocks workgroups of 256 threads.
 * kind 0 read src (dst receives n_blocks partial sums, so dst must hold
 * n_blocks floats), 1 write dst, 2 copy src to dst.  nt != 0: non-temporal
 * loads and stores.  bytes a positive multiple of 16, pointers 16-byte
 * aligned; otherwise RMDF_E_INVAL.  Timing is the caller's (events around the
 * call).  Gives the practical ceiling beside the data-sheet HBM peak. */
rmdf_status rmdf_hbm_probe(int kind, const void *src, void *dst, size_t bytes, int n_blocks, int nt, void *stream);

/* Bytes of device memory the context holds. */
rmdf_status rmdf_device_bytes(const rmdf_ctx *ctx, size_t *bytes);

/* ---- Checkpoint and restore ---------------------------------------------
 * The filter is recursive in time (Sec. 1): all it carries from frame to
 * frame is the observer state (or, in the temporal ring and direct forms,
 * the ring of the last Kt 2-D spectra), the smoothed autocorrelation R'
 * (Sec. 2, eq. 9-10 with the exponential smoother), the delay ring of raw
 * frames (eq. 1 and 4 read the frame m'_t back), the frame count and the
 * non-finite counter.  A saved state holds exactly these, plus the latest
 * output, velocity and index (so the readouts after a restore equal those
 * before the save), behind a 128-byte header naming the context's shape.
 * The learned mode's features and network outputs are not part of it (they
 * are recomputed by the next push); its weights are set separately.
 *
 * rmdf_state_bytes: size of a saved state of this context.
 * rmdf_save_state: writes it to buf (host or device memory, at least
 *   rmdf_state_bytes bytes, owned by the caller); ordered after the pushes
 *   already queued on the context stream; returns when the copy is complete.
 *   Errors: RMDF_E_INVAL (NULL, buffer too small), RMDF_E_DEVICE.
 * rmdf_load_state: replaces the context's state by one saved from a context
 *   created with the same frame size, window, candidate grid (values, not
 *   only sizes), parameters (B, m', alpha, velocity mode, fixed velocity,
 *   kernel variant, temporal form); the next push continues that stream bit
 *   for bit as the saved context would have.  Returns when the copy is
 *   complete.  Errors: RMDF_E_INVAL (NULL, short buffer, not a saved state,
 *   or saved from a different configuration; the context is then unchanged),
 *   RMDF_E_STATE (a stream owned by a batch), RMDF_E_DEVICE.
 * Because the observer is deadbeat, a state whose spectrum part is damaged
 * (any finite values) is flushed exactly after Kt pushes in exact arithmetic;
 * the smoothed R then forgets it geometrically (factor alpha per frame). */
rmdf_status rmdf_state_bytes(const rmdf_ctx *ctx, size_t *bytes);
rmdf_status rmdf_save_state(rmdf_ctx *ctx, void *buf, size_t bytes);
rmdf_status rmdf_load_state(rmdf_ctx *ctx, const void *buf, size_t bytes);

/* Free everything; ctx may be NULL. */
rmdf_status rmdf_destroy(rmdf_ctx *ctx);

/* ---- Many streams in one step -------------------------------------------
 * Independent sensor streams, each with its own frame size, window and
 * candidate grid, advanced together one frame per step.  A step is one
 * hipGraph launch of two kernels: the row sliding DFT of every stream, then a
 * persistent per-pixel kernel whose workgroups pull (stream, tile) items from
 * a queue ordered by decreasing cost.  Window shapes and velocity modes as for
 * rmdf_create (search or fixed). */
typedef struct rmdf_batch rmdf_batch;
typedef struct {
  int H, W, Kx, Ky, Kt;              /* frame size and window lengths         */
  const float *vgrid_x, *vgrid_y;    /* host candidate grids (copied)         */
  int nvx, nvy;
} rmdf_stream_desc;

/* Create n streams (p applies to all; NULL: defaults).  hip_stream: stream to
 * run on; NULL creates one (a captured graph cannot run on the null stream).
 * Errors as rmdf_create, reported for the first failing stream;
 * RMDF_E_UNSUPPORTED for a velocity mode other than search or fixed, a
 * temporal form other than the observer, or write_features. */
rmdf_status rmdf_batch_create(int n, const rmdf_stream_desc *streams, const rmdf_params *p,
                              void *hip_stream, rmdf_batch **out);
/* Device address where the next frame of stream s (H*W FP32) must be written
 * before rmdf_batch_launch (zero-copy input).  The write must be complete, or
 * ordered before the launch on the batch's stream, when the launch is made:
 * the batch stream does not wait for work on other streams (a device-to-device
 * hipMemcpy may return before the copy has finished). */
rmdf_status rmdf_batch_input(rmdf_batch *b, int s, float **frame_dev);
/* Advance every stream by one frame (one graph launch). */
rmdf_status rmdf_batch_launch(rmdf_batch *b);
/* Copy frames_dev[s] (n device pointers) into the input slots, then launch. */
rmdf_status rmdf_batch_push(rmdf_batch *b, const float *const *frames_dev);
/* Latest output / velocity / index of stream s (any may be NULL). */
rmdf_status rmdf_batch_output(rmdf_batch *b, int s, float *out_dev, float *vxy_dev, int *idx_dev);
/* The single-stream view of stream s (for rmdf_spectrum, rmdf_smoothed_r...);
 * owned by the batch, do not destroy it or push frames through it. */
rmdf_status rmdf_batch_stream_ctx(rmdf_batch *b, int s, rmdf_ctx **ctx);
/* Rows per work tile for stream s (s = -1: all); rebuilds the graph. */
rmdf_status rmdf_batch_set_tiles(rmdf_batch *b, int s, int tile_rows);
/* Schedule of the per-pixel tiles within a step; rebuilds the graph.
 * 0 (default): one persistent kernel per tile family, largest family first;
 * 1: one persistent kernel for the 16x16x8 wave-per-anchor, 8x8x4 and 9x9x5
 *    families, their work items interleaved in proportion;
 * 2: as 0, with the 8x8x4 and 9x9x5 kernels on a parallel branch of the
 *    graph (they may run beside the 16x16x8 kernel);
 * 3: as 2, the parallel branch's kernels launched first.
 * Other values: RMDF_E_INVAL.  The results do not depend on the schedule.
 * The autotuner tries all four. */
rmdf_status rmdf_batch_set_schedule(rmdf_batch *b, int schedule);
/* Pick rows per tile for each size class and the persistent grid size by
 * timing whole steps (iters timed launches per candidate).  The streams
 * advance while tuning (whatever the input slots hold is consumed).  A text
 * summary goes to report (may be NULL). */
rmdf_status rmdf_batch_autotune(rmdf_batch *b, int iters, char *report, size_t report_len);
/* Per-step latency (HIP events around each graph launch while timing is on):
 * median, 99th percentile and mean in ms over the launches since the last
 * call; synchronises the stream. */
rmdf_status rmdf_batch_set_timing(rmdf_batch *b, int on);
rmdf_status rmdf_batch_latency(rmdf_batch *b, float *p50_ms, float *p99_ms, float *mean_ms, long long *n);
rmdf_status rmdf_batch_destroy(rmdf_batch *b);
const char *rmdf_batch_last_error(const rmdf_batch *b);

/* Message of the last error on ctx (NULL ctx: the calling thread's last
 * rmdf_create error).  Never NULL. */
const char *rmdf_last_error(const rmdf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* RMDF_H */
