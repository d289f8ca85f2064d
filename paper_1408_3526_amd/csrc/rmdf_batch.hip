// rmdf_batch.hip - many independent sensor streams (uneven frame sizes and
// windows) advanced one frame per step by the kernels of one hipGraph:
//   k_row_batch          row sliding DFT of every stream (one block per
//                        (stream, row, chunk)); reads each stream's raw frame
//                        from its delay-ring slot, non-finite samples read as 0
//   k_batch_tiles<KIND>  persistent workgroups pull (stream, tile) items of one
//                        tile family (8x8x4, 9x9x5, generic 16x16x8, 16x16x8
//                        wave-per-anchor) from an atomic queue ordered by
//                        decreasing cost and run that stream's per-pixel tile;
//                        one kernel per family, each with its own register
//                        budget (the default schedule)
//   k_batch_mixed        the alternative schedule: one persistent kernel whose
//                        single queue interleaves the wave-per-anchor, 8x8x4
//                        and 9x9x5 tiles
//   k_batch_advance      advances every stream's frame counter and re-arms the
//                        queues for the next step
// Nothing in the graph changes between steps: frame counters live in device
// memory and frames are written into the ring slots before each launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rmdf.h"
#include "rmdf_device.h"
#include "rmdf_internal.h"
#include "rmdf_pixel16.h"

namespace rmdf {

enum : int { KIND_884 = 0, KIND_995 = 1, KIND_16G = 2, KIND_16W = 3, NKIND = 4 };

struct RowDesc {
  const float* ring;                 // stream's delay ring
  float2* rs;                        // row spectra
  const float2* twx;
  unsigned long long* nonfinite;
  long long hw;                      // H * W
  int H, W, MX, nring;
  int chunks;                        // row chunks per row
  int item_base;                     // first block index of this stream
};

struct BatchPixDesc {
  PixArgs a;                         // static fields; ring_delayed filled per step
  const float* ring;
  long long hw;
  int nring, dt, kind;
};

struct BatchState {
  long long* t;                      // [n] frames pushed per stream (device)
  unsigned int* queue;               // [NKIND] next work item of each tile family
};

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t ROW_SMEM = cmax(cmax(RowShape<8>::SMEM, RowShape<16>::SMEM), RowShape<9>::SMEM);

__global__ void __launch_bounds__(256) k_row_batch(const RowDesc* __restrict__ d, int n, const long long* __restrict__ t) {
  __shared__ __align__(16) char smem[ROW_SMEM];
  int s = 0;
  while (s + 1 < n && (int)blockIdx.x >= d[s + 1].item_base) ++s;   // wave-uniform scan (n is small)
  const RowDesc& r = d[s];
  const int local = blockIdx.x - r.item_base;
  const int y = local / r.chunks, x0 = (local % r.chunks) * RCX;
  const float* f = r.ring + (size_t)(t[s] % r.nring) * r.hw;
  if (r.MX == 8) row_chunk<8>(f, r.rs, r.twx, r.H, r.W, y, x0, smem, r.nonfinite);
  else if (r.MX == 16) row_chunk<16>(f, r.rs, r.twx, r.H, r.W, y, x0, smem, r.nonfinite);
  else row_chunk<9>(f, r.rs, r.twx, r.H, r.W, y, x0, smem, r.nonfinite);
}

// Item loop shared by both persistent kernels: claim the next item, run its
// tile, until the family's queue is empty.
template <class F>
static __device__ void item_loop(const BatchPixDesc* __restrict__ d, const int4* __restrict__ items, int n_items,
                                 unsigned int* queue, const long long* t, unsigned int* s_item, F&& run) {
  for (;;) {
    if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1u);
    __syncthreads();
    // uniform: the item's descriptor then lives in scalar registers
    const unsigned int it = __builtin_amdgcn_readfirstlane(*s_item);
    __syncthreads();                    // all have read s_item before it is overwritten
    if (it >= (unsigned int)n_items) break;
    const int4 w = items[it];
    const BatchPixDesc& bd = d[w.x];
    const long long tt = t[w.x];
    const float* rd = (tt >= bd.dt) ? bd.ring + (size_t)((tt - bd.dt) % bd.nring) * bd.hw : nullptr;
    run(bd, rd, w);
  }
}

template <int KIND> struct KindSmem;
template <> struct KindSmem<KIND_884> { static constexpr size_t v = Shape<8, 8, 4>::SMEM; };
template <> struct KindSmem<KIND_995> { static constexpr size_t v = Shape<9, 9, 5>::SMEM; };
template <> struct KindSmem<KIND_16G> { static constexpr size_t v = Shape<16, 16, 8>::SMEM; };
template <> struct KindSmem<KIND_16W> { static constexpr size_t v = p16::SMEM16; };

// One persistent kernel per tile family (its queue is queue[KIND]), so every
// tile keeps its own register budget; the 16x16x8 wave-per-anchor tile runs
// two workgroups per CU, as in the single-stream kernel.
template <int KIND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KIND == KIND_16W ? 2 : 1)))
k_batch_tiles(const BatchPixDesc* __restrict__ d, const int4* __restrict__ items, int n_items, BatchState bs) {
  __shared__ __align__(16) char smem[KindSmem<KIND>::v];
  __shared__ unsigned int s_item;
  item_loop(d, items, n_items, bs.queue + KIND, bs.t, &s_item, [&](const BatchPixDesc& bd, const float* rd, int4 w) {
    if (KIND == KIND_884) pixel_tile<8, 8, 4>(bd.a, rd, w.y, w.z, smem);
    else if (KIND == KIND_995) pixel_tile<9, 9, 5>(bd.a, rd, w.y, w.z, smem);
    else if (KIND == KIND_16G) pixel_tile<16, 16, 8>(bd.a, rd, w.y, w.z, smem);
    else p16::pixel16_tile<0>(bd.a, rd, w.y, w.z, smem);
  });
}

// One persistent kernel for the wave-per-anchor 16x16x8 tiles and the 8x8x4
// and 9x9x5 tiles: a single queue (queue[0]) whose items interleave the
// families in proportion, so the small, latency-bound tiles run beside the
// memory-bound 16x16x8 ones instead of after them.  Register budget of the
// largest tile (two workgroups per CU), LDS of the largest family.  The
// generic 16x16x8 tile keeps its own kernel (its register demand would push
// this one into scratch).
constexpr size_t MIXED_SMEM = cmax(cmax(KindSmem<KIND_884>::v, KindSmem<KIND_995>::v), KindSmem<KIND_16W>::v);
constexpr bool in_mixed(int kind) { return kind != KIND_16G; }

// The small tiles are called rather than inlined into the mixed kernel: each
// keeps its own register allocation, and the 16x16x8 path (inlined) keeps its
// registers free of spills.
static __device__ __attribute__((noinline)) void tile884(const PixArgs& a, const float* rd, int xb, int yb, char* smem) {
  pixel_tile<8, 8, 4>(a, rd, xb, yb, smem);
}
static __device__ __attribute__((noinline)) void tile995(const PixArgs& a, const float* rd, int xb, int yb, char* smem) {
  pixel_tile<9, 9, 5>(a, rd, xb, yb, smem);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_mixed(const BatchPixDesc* __restrict__ d, const int4* __restrict__ items, int n_items, BatchState bs) {
  __shared__ __align__(16) char smem[MIXED_SMEM];
  __shared__ unsigned int s_item;
  item_loop(d, items, n_items, bs.queue, bs.t, &s_item, [&](const BatchPixDesc& bd, const float* rd, int4 w) {
    const int kind = __builtin_amdgcn_readfirstlane(bd.kind);
    if (kind == KIND_16W) p16::pixel16_tile<0>(bd.a, rd, w.y, w.z, smem);
    else if (kind == KIND_884) tile884(bd.a, rd, w.y, w.z, smem);
    else tile995(bd.a, rd, w.y, w.z, smem);
  });
}

// End of a step: every stream has consumed one frame; re-arm the queues (a
// kernel, not a memset, so the same code is safe to capture).
__global__ void k_batch_advance(BatchState bs, int n_streams) {
  for (int s = threadIdx.x; s < n_streams; s += blockDim.x) bs.t[s] += 1;
  if (threadIdx.x < NKIND) bs.queue[threadIdx.x] = 0u;
}

// Zeroes the queues before the first step.
__global__ void k_batch_arm(BatchState bs) {
  if (threadIdx.x < NKIND) bs.queue[threadIdx.x] = 0u;
}

}  // namespace rmdf

using namespace rmdf;

struct rmdf_batch {
  int n = 0;
  std::vector<rmdf_ctx*> ctx;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<int> tile_rows;        // per stream
  int grid_mult = 1;                 // persistent workgroups per resident slot
  // schedule of the pixel tiles: 0 one kernel per family, one after another;
  // 1 one kernel for all families (k_batch_mixed); 2 one kernel per family,
  // the small families on a second graph branch beside the 16x16x8 kernels;
  // 3 as 2, the small families' kernels launched first
  int schedule = 0;
  int mixed_blocks = 0;
  hipStream_t side = nullptr;        // second capture stream (schedules 2, 3)
  hipEvent_t fork = nullptr, join = nullptr;
  // device
  RowDesc* d_row = nullptr;
  BatchPixDesc* d_pix = nullptr;
  int4* d_items = nullptr;
  long long* d_t = nullptr;
  unsigned int* d_queue = nullptr;   // [NKIND]
  int row_blocks = 0;
  int n_items[NKIND] = {};           // work items of each tile family
  int blocks[NKIND] = {};            // persistent workgroups of each family's kernel
  std::vector<long long> t;          // host mirror of the frame counters
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<float> lat_ms;
  std::string err;
};

static rmdf_status bfail(rmdf_batch* b, rmdf_status s, const std::string& m) {
  if (b) b->err = m;
  else rmdf_internal_set_create_error(m);
  return s;
}

static int kind_of(const rmdf_ctx* c) {
  int mx, my, mz, variant;
  rmdf_internal_shape(c, &mx, &my, &mz, &variant);
  if (mx == 8) return KIND_884;
  if (mx == 9) return KIND_995;
  return variant == 2 ? KIND_16W : KIND_16G;
}

static void free_graph(rmdf_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Work items and the captured graph for the current tile choice.
static hipError_t rebuild(rmdf_batch* b) {
  hipError_t e;
  free_graph(b);
  struct Item { int4 w; double cost; };
  std::vector<Item> items;
  std::vector<BatchPixDesc> pd(b->n);
  for (int s = 0; s < b->n; ++s) {
    rmdf_ctx* c = b->ctx[s];
    PixArgs a = rmdf_internal_pixargs(c);
    a.TY = b->tile_rows[s];
    BatchPixDesc& d = pd[s];
    d.a = a;
    d.kind = kind_of(c);
    d.ring = rmdf_internal_ring(c, &d.nring, &d.dt);
    d.hw = (long long)a.H * a.W;
    const int cols = (d.kind == KIND_16W) ? 4 : (d.kind == KIND_884 ? 8 : (d.kind == KIND_995 ? 4 : 2));
    const int xblocks = (a.W + cols - 1) / cols, yblocks = (a.H + a.TY - 1) / a.TY;
    int mx, my, mz, v;
    rmdf_internal_shape(c, &mx, &my, &mz, &v);
    const double per_px = 8.0 * mx * my * mz + 8.0 * a.nv;
    for (int yb = 0; yb < yblocks; ++yb)
      for (int xb = 0; xb < xblocks; ++xb) {
        const int rows = std::min(a.TY, a.H - yb * a.TY), colsn = std::min(cols, a.W - xb * cols);
        items.push_back({make_int4(s, xb, yb, 0), per_px * rows * colsn});
      }
  }
  // grouped by tile family, each group longest first so the tail of its
  // kernel is made of small items
  std::stable_sort(items.begin(), items.end(), [&](const Item& p, const Item& q) {
    const int fp = pd[p.w.x].kind, fq = pd[q.w.x].kind;
    if (fp != fq) return fp < fq;
    return p.cost > q.cost;
  });
  std::vector<int4> iv(items.size());
  for (int k = 0; k < NKIND; ++k) b->n_items[k] = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    iv[i] = items[i].w;
    b->n_items[pd[items[i].w.x].kind] += 1;
  }
  int n_mixed = 0;
  const bool mixed = (b->schedule == 1);
  if (mixed) {
    // the generic 16x16x8 items keep their family's place; the others are
    // interleaved: item j of a family with n items sits at (j + 1/2) / n of
    // the mixed queue, so every family advances at the same relative rate and
    // the queue still ends with each family's smallest items
    std::vector<std::pair<double, int4>> keyed;
    int first = 0;
    for (int k = 0; k < NKIND; ++k) {
      if (in_mixed(k))
        for (int j = 0; j < b->n_items[k]; ++j) keyed.push_back({(j + 0.5) / b->n_items[k], iv[first + j]});
      first += b->n_items[k];
    }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const std::pair<double, int4>& p, const std::pair<double, int4>& q) { return p.first < q.first; });
    // layout: [generic 16x16x8 items][mixed items]
    std::vector<int4> jv;
    jv.reserve(iv.size());
    first = 0;
    for (int k = 0; k < NKIND; ++k) {
      if (!in_mixed(k))
        for (int j = 0; j < b->n_items[k]; ++j) jv.push_back(iv[first + j]);
      first += b->n_items[k];
    }
    for (auto& kv : keyed) jv.push_back(kv.second);
    iv.swap(jv);
    n_mixed = (int)keyed.size();
  }
  if (b->d_items) hipFree(b->d_items);
  b->d_items = nullptr;
  if ((e = hipMalloc(&b->d_items, sizeof(int4) * std::max<size_t>(iv.size(), 1))) != hipSuccess) return e;
  if ((e = hipMemcpy(b->d_items, iv.data(), sizeof(int4) * iv.size(), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(b->d_pix, pd.data(), sizeof(BatchPixDesc) * b->n, hipMemcpyHostToDevice)) != hipSuccess) return e;

  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void* kern[NKIND] = {reinterpret_cast<const void*>(k_batch_tiles<KIND_884>),
                             reinterpret_cast<const void*>(k_batch_tiles<KIND_995>),
                             reinterpret_cast<const void*>(k_batch_tiles<KIND_16G>),
                             reinterpret_cast<const void*>(k_batch_tiles<KIND_16W>)};
  for (int k = 0; k < NKIND; ++k) {
    int occ = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern[k], 256, 0);
    b->blocks[k] = std::min(b->n_items[k], cus * std::max(occ, 1) * b->grid_mult);
  }
  {
    int occ = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_batch_mixed), 256, 0);
    b->mixed_blocks = std::min(n_mixed, cus * std::max(occ, 1) * b->grid_mult);
  }

  BatchState bs{b->d_t, b->d_queue};
  if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_batch, dim3(b->row_blocks), dim3(256), 0, b->stream, b->d_row, b->n,
                     (const long long*)b->d_t);
  if (mixed && b->mixed_blocks > 0)
    hipLaunchKernelGGL(k_batch_mixed, dim3(b->mixed_blocks), dim3(256), 0, b->stream, b->d_pix,
                       (const int4*)b->d_items + (iv.size() - n_mixed), n_mixed, bs);
  // schedules 2 and 3: fork after the row pass, the small families on the
  // side branch (3: captured, hence dispatched, before the large families, so
  // their workgroups are resident first and the 16x16x8 kernel's persistent
  // workgroups take their slots as they finish)
  const bool branch = (b->schedule >= 2) && (b->blocks[KIND_884] > 0 || b->blocks[KIND_995] > 0);
  if (branch) {
    hipEventRecord(b->fork, b->stream);
    hipStreamWaitEvent(b->side, b->fork, 0);
  }
  // per family: the largest tiles first (in mixed mode only the generic
  // 16x16x8 family, whose items open the list, on queue[KIND_16G])
  static const int largest_first[NKIND] = {KIND_16W, KIND_16G, KIND_995, KIND_884};
  static const int small_first[NKIND] = {KIND_995, KIND_884, KIND_16W, KIND_16G};
  const int* order = (branch && b->schedule == 3) ? small_first : largest_first;
  for (int i = 0; i < NKIND; ++i) {
    const int k = order[i];
    if ((mixed && in_mixed(k)) || b->blocks[k] == 0) continue;
    int first = 0;
    if (!mixed)
      for (int j = 0; j < k; ++j) first += b->n_items[j];
    const int4* it = (const int4*)b->d_items + first;
    const hipStream_t st = (branch && (k == KIND_884 || k == KIND_995)) ? b->side : b->stream;
    switch (k) {
      case KIND_884: hipLaunchKernelGGL(k_batch_tiles<KIND_884>, dim3(b->blocks[k]), dim3(256), 0, st, b->d_pix, it, b->n_items[k], bs); break;
      case KIND_995: hipLaunchKernelGGL(k_batch_tiles<KIND_995>, dim3(b->blocks[k]), dim3(256), 0, st, b->d_pix, it, b->n_items[k], bs); break;
      case KIND_16G: hipLaunchKernelGGL(k_batch_tiles<KIND_16G>, dim3(b->blocks[k]), dim3(256), 0, st, b->d_pix, it, b->n_items[k], bs); break;
      default: hipLaunchKernelGGL(k_batch_tiles<KIND_16W>, dim3(b->blocks[k]), dim3(256), 0, st, b->d_pix, it, b->n_items[k], bs); break;
    }
  }
  if (branch) {
    hipEventRecord(b->join, b->side);
    hipStreamWaitEvent(b->stream, b->join, 0);
  }
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(256), 0, b->stream, bs, b->n);
  if ((e = hipStreamEndCapture(b->stream, &b->graph)) != hipSuccess) return e;
  if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) return e;
  return hipSuccess;
}

extern "C" {

rmdf_status rmdf_batch_create(int n, const rmdf_stream_desc* sd, const rmdf_params* p, void* hip_stream,
                              rmdf_batch** out) {
  if (!out) return bfail(nullptr, RMDF_E_INVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > 4096 || !sd) return bfail(nullptr, RMDF_E_INVAL, "need 1..4096 stream descriptors");
  rmdf_batch* b = new rmdf_batch();
  b->n = n;
  hipError_t e;
  if (hip_stream) {
    b->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    // graph capture needs a real stream (the null stream cannot be captured)
    if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) {
      delete b;
      return bfail(nullptr, RMDF_E_DEVICE, "stream creation failed");
    }
    b->own_stream = true;
  }
  auto bail = [&](rmdf_status st, const std::string& m) {
    for (auto* c : b->ctx) rmdf_destroy(c);
    if (b->side) hipStreamDestroy(b->side);
    if (b->fork) hipEventDestroy(b->fork);
    if (b->join) hipEventDestroy(b->join);
    if (b->own_stream) hipStreamDestroy(b->stream);
    delete b;
    return bfail(nullptr, st, m);
  };
  if (p && p->velocity_mode != RMDF_VEL_SEARCH && p->velocity_mode != RMDF_VEL_FIXED)
    return bail(RMDF_E_UNSUPPORTED, "batched streams support the search and fixed velocity modes");
  if (p && p->temporal != RMDF_TEMPORAL_OBSERVER)
    return bail(RMDF_E_UNSUPPORTED, "batched streams use the observer state (temporal mode 0)");
  if (p && p->write_features)
    return bail(RMDF_E_UNSUPPORTED, "batched streams do not write the learned model's features");
  std::vector<RowDesc> rd(n);
  int base = 0;
  for (int s = 0; s < n; ++s) {
    rmdf_ctx* c = nullptr;
    rmdf_status st = rmdf_create(sd[s].H, sd[s].W, sd[s].Kx, sd[s].Ky, sd[s].Kt, sd[s].vgrid_x, sd[s].nvx,
                                 sd[s].vgrid_y, sd[s].nvy, p, b->stream, &c);
    if (st != RMDF_OK) return bail(st, std::string("stream ") + std::to_string(s) + ": " + rmdf_last_error(nullptr));
    rmdf_internal_set_batch_owned(c);
    b->ctx.push_back(c);
    PixArgs a = rmdf_internal_pixargs(c);
    b->tile_rows.push_back(a.TY);
    int nring, dt;
    RowDesc& r = rd[s];
    r.ring = rmdf_internal_ring(c, &nring, &dt);
    r.nring = nring;
    r.rs = const_cast<float2*>(a.rs);
    r.twx = rmdf_internal_twx(c);
    r.nonfinite = rmdf_internal_nonfinite(c);
    r.H = a.H;
    r.W = a.W;
    int mx, my, mz, v;
    rmdf_internal_shape(c, &mx, &my, &mz, &v);
    r.MX = mx;
    r.hw = (long long)a.H * a.W;
    r.chunks = (a.W + RCX - 1) / RCX;
    r.item_base = base;
    base += r.chunks * a.H;
  }
  b->row_blocks = base;
  // second branch of the captured step (schedules 2, 3); default priority
  if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess)
    return bail(RMDF_E_DEVICE, "stream or event creation failed");
  b->t.assign(n, 0);
  if ((e = hipMalloc(&b->d_row, sizeof(RowDesc) * n)) != hipSuccess) return bail(RMDF_E_NOMEM, "descriptors");
  if ((e = hipMalloc(&b->d_pix, sizeof(BatchPixDesc) * n)) != hipSuccess) return bail(RMDF_E_NOMEM, "descriptors");
  if ((e = hipMalloc(&b->d_t, sizeof(long long) * n)) != hipSuccess) return bail(RMDF_E_NOMEM, "counters");
  if ((e = hipMalloc(&b->d_queue, NKIND * sizeof(unsigned int))) != hipSuccess) return bail(RMDF_E_NOMEM, "counters");
  if ((e = hipMemcpy(b->d_row, rd.data(), sizeof(RowDesc) * n, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_t, b->t.data(), sizeof(long long) * n, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(RMDF_E_DEVICE, std::string("descriptor upload: ") + hipGetErrorString(e));
  hipLaunchKernelGGL(k_batch_arm, dim3(1), dim3(64), 0, b->stream, BatchState{b->d_t, b->d_queue});
  if ((e = rebuild(b)) != hipSuccess) return bail(RMDF_E_DEVICE, std::string("graph: ") + hipGetErrorString(e));
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return bail(RMDF_E_DEVICE, "sync");
  *out = b;
  return RMDF_OK;
}

rmdf_status rmdf_batch_input(rmdf_batch* b, int s, float** frame_dev) {
  if (!b || !frame_dev || s < 0 || s >= b->n) return bfail(b, RMDF_E_INVAL, "bad arguments");
  int nring, dt;
  float* ring = const_cast<float*>(rmdf_internal_ring(b->ctx[s], &nring, &dt));
  const PixArgs a = rmdf_internal_pixargs(b->ctx[s]);
  *frame_dev = ring + (size_t)(b->t[s] % nring) * (size_t)a.H * a.W;
  return RMDF_OK;
}

rmdf_status rmdf_batch_launch(rmdf_batch* b) {
  if (!b) return bfail(nullptr, RMDF_E_INVAL, "batch is NULL");
  hipError_t e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (b->timing) {
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipEventRecord(e0, b->stream);
  }
  if ((e = hipGraphLaunch(b->exec, b->stream)) != hipSuccess) return bfail(b, RMDF_E_DEVICE, hipGetErrorString(e));
  if (b->timing) {
    hipEventRecord(e1, b->stream);
    b->ev.emplace_back(e0, e1);
  }
  for (int s = 0; s < b->n; ++s) {
    b->t[s] += 1;
    rmdf_internal_advance(b->ctx[s]);
  }
  return RMDF_OK;
}

rmdf_status rmdf_batch_push(rmdf_batch* b, const float* const* frames) {
  if (!b || !frames) return bfail(b, RMDF_E_INVAL, "bad arguments");
  for (int s = 0; s < b->n; ++s) {
    if (!frames[s]) return bfail(b, RMDF_E_INVAL, "NULL frame pointer");
    float* dst = nullptr;
    rmdf_batch_input(b, s, &dst);
    const PixArgs a = rmdf_internal_pixargs(b->ctx[s]);
    hipError_t e = hipMemcpyAsync(dst, frames[s], sizeof(float) * (size_t)a.H * a.W, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return bfail(b, RMDF_E_DEVICE, hipGetErrorString(e));
  }
  return rmdf_batch_launch(b);
}

rmdf_status rmdf_batch_output(rmdf_batch* b, int s, float* out, float* vxy, int* idx) {
  if (!b || s < 0 || s >= b->n) return bfail(b, RMDF_E_INVAL, "bad arguments");
  rmdf_status st = RMDF_OK;
  if (out) st = rmdf_output(b->ctx[s], out);
  if (st == RMDF_OK && (vxy || idx)) st = rmdf_velocity(b->ctx[s], vxy, idx);
  if (st != RMDF_OK) return bfail(b, st, rmdf_last_error(b->ctx[s]));
  return RMDF_OK;
}

rmdf_status rmdf_batch_stream_ctx(rmdf_batch* b, int s, rmdf_ctx** ctx) {
  if (!b || !ctx || s < 0 || s >= b->n) return bfail(b, RMDF_E_INVAL, "bad arguments");
  *ctx = b->ctx[s];
  return RMDF_OK;
}

rmdf_status rmdf_batch_set_tiles(rmdf_batch* b, int s, int tile_rows) {
  if (!b || s < -1 || s >= b->n || tile_rows < 1) return bfail(b, RMDF_E_INVAL, "bad arguments");
  hipStreamSynchronize(b->stream);
  for (int i = 0; i < b->n; ++i)
    if (s < 0 || i == s) b->tile_rows[i] = tile_rows;
  hipError_t e = rebuild(b);
  if (e != hipSuccess) return bfail(b, RMDF_E_DEVICE, hipGetErrorString(e));
  return RMDF_OK;
}

rmdf_status rmdf_batch_set_schedule(rmdf_batch* b, int schedule) {
  if (!b || schedule < 0 || schedule > 3) return bfail(b, RMDF_E_INVAL, "schedule must be 0, 1, 2 or 3");
  hipStreamSynchronize(b->stream);
  b->schedule = schedule;
  hipError_t e = rebuild(b);
  if (e != hipSuccess) return bfail(b, RMDF_E_DEVICE, hipGetErrorString(e));
  return RMDF_OK;
}

rmdf_status rmdf_batch_set_timing(rmdf_batch* b, int on) {
  if (!b) return bfail(nullptr, RMDF_E_INVAL, "batch is NULL");
  b->timing = on != 0;
  return RMDF_OK;
}

static void collect(rmdf_batch* b) {
  hipStreamSynchronize(b->stream);
  for (auto& pr : b->ev) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, pr.first, pr.second);
    b->lat_ms.push_back(ms);
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  b->ev.clear();
}

rmdf_status rmdf_batch_latency(rmdf_batch* b, float* p50, float* p99, float* mean, long long* n) {
  if (!b || !p50 || !p99 || !mean || !n) return bfail(b, RMDF_E_INVAL, "bad arguments");
  collect(b);
  std::vector<float> v = b->lat_ms;
  b->lat_ms.clear();
  *n = (long long)v.size();
  if (v.empty()) { *p50 = *p99 = *mean = 0.f; return RMDF_OK; }
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)std::floor(q * (v.size() - 1) + 0.5))]; };
  *p50 = pct(0.50);
  *p99 = pct(0.99);
  double s = 0;
  for (float x : v) s += x;
  *mean = (float)(s / v.size());
  return RMDF_OK;
}

// Coordinate descent over the rows per work tile of each size class (streams
// with the same frame size and window), timing whole steps; the frames in the
// input slots are consumed (the streams advance).
rmdf_status rmdf_batch_autotune(rmdf_batch* b, int iters, char* report, size_t report_len) {
  if (!b || iters < 1) return bfail(b, RMDF_E_INVAL, "bad arguments");
  struct Cls { int H, W, kind; std::vector<int> members; };
  std::vector<Cls> cls;
  for (int s = 0; s < b->n; ++s) {
    const PixArgs a = rmdf_internal_pixargs(b->ctx[s]);
    const int k = kind_of(b->ctx[s]);
    auto it = std::find_if(cls.begin(), cls.end(), [&](const Cls& c) { return c.H == a.H && c.W == a.W && c.kind == k; });
    if (it == cls.end()) cls.push_back({a.H, a.W, k, {s}});
    else it->members.push_back(s);
  }
  const bool was = b->timing;
  auto measure = [&]() -> float {
    b->timing = true;
    collect(b);
    b->lat_ms.clear();
    for (int i = 0; i < 2; ++i) rmdf_batch_launch(b);   // warm
    collect(b);
    b->lat_ms.clear();
    for (int i = 0; i < iters; ++i) rmdf_batch_launch(b);
    collect(b);
    std::vector<float> v = b->lat_ms;
    b->lat_ms.clear();
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
  };
  const int cand[] = {8, 16, 32, 64};
  std::string rep;
  float best_all = measure();
  for (auto& c : cls) {
    int best_ty = b->tile_rows[c.members[0]];
    for (int ty : cand) {
      if (ty == best_ty) continue;
      for (int s : c.members) b->tile_rows[s] = ty;
      if (rebuild(b) != hipSuccess) return bfail(b, RMDF_E_DEVICE, "rebuild failed");
      const float m = measure();
      if (m < best_all) { best_all = m; best_ty = ty; }
    }
    for (int s : c.members) b->tile_rows[s] = best_ty;
    if (rebuild(b) != hipSuccess) return bfail(b, RMDF_E_DEVICE, "rebuild failed");
    char line[160];
    std::snprintf(line, sizeof line, "%dx%d kind %d (%zu streams): tile_rows %d\n", c.W, c.H, c.kind,
                  c.members.size(), best_ty);
    rep += line;
  }
  int best_mult = b->grid_mult;
  for (int m : {1, 2}) {
    if (m == best_mult) continue;
    b->grid_mult = m;
    if (rebuild(b) != hipSuccess) return bfail(b, RMDF_E_DEVICE, "rebuild failed");
    const float t = measure();
    if (t < best_all) { best_all = t; best_mult = m; }
  }
  b->grid_mult = best_mult;
  // schedule of the tile families
  int best_sched = b->schedule;
  for (int sc = 0; sc < 4; ++sc) {
    if (sc == best_sched) continue;
    b->schedule = sc;
    if (rebuild(b) != hipSuccess) return bfail(b, RMDF_E_DEVICE, "rebuild failed");
    const float t = measure();
    if (t < best_all) { best_all = t; best_sched = sc; }
  }
  b->schedule = best_sched;
  if (rebuild(b) != hipSuccess) return bfail(b, RMDF_E_DEVICE, "rebuild failed");
  static const char* sched_name[4] = {"one kernel per tile family", "one kernel for all tile families",
                                      "one kernel per tile family, small families on a parallel branch",
                                      "one kernel per tile family, small families first on a parallel branch"};
  char line[200];
  std::snprintf(line, sizeof line, "persistent workgroups per slot %d; %s; median step %.3f ms\n", best_mult,
                sched_name[b->schedule], best_all);
  rep += line;
  b->timing = was;
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return RMDF_OK;
}

rmdf_status rmdf_batch_destroy(rmdf_batch* b) {
  if (!b) return RMDF_OK;
  hipStreamSynchronize(b->stream);
  for (auto& pr : b->ev) { hipEventDestroy(pr.first); hipEventDestroy(pr.second); }
  free_graph(b);
  if (b->side) hipStreamDestroy(b->side);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->join) hipEventDestroy(b->join);
  hipFree(b->d_items);
  hipFree(b->d_row);
  hipFree(b->d_pix);
  hipFree(b->d_t);
  hipFree(b->d_queue);
  for (auto* c : b->ctx) rmdf_destroy(c);
  if (b->own_stream) hipStreamDestroy(b->stream);
  delete b;
  return RMDF_OK;
}

const char* rmdf_batch_last_error(const rmdf_batch* b) {
  if (!b) return rmdf_last_error(nullptr);
  return b->err.c_str();
}

}  // extern "C"
