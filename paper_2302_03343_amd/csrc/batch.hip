// Batched VEGAS: many independent integrals of uneven dimension and sample
// count in one persistent launch per iteration, captured with the
// reductions and the refinements in one HIP graph.
//
// Each integral keeps its own grid, Philox stream and record list (its
// vgx_vegas context), so an integral computed in a batch draws exactly the
// samples it would draw alone (thesis VEGAS section for the per-integral
// algorithm; the batching is an implementation choice).
//
// MI355X design
//   * work is cut into tiles of T consecutive samples of one integral; the
//     tiles of all integrals form one index space, integral i owning the
//     range [tile0_i, tile0_i + ntiles_i);
//   * a persistent grid (as many workgroups as can be resident at once)
//     pops tile indices from an atomic counter, so integrals with 1e4 and
//     1e7 samples load-balance across the 256 CUs; a workgroup re-stages the
//     grid edges in LDS only when the integral changes between its tiles;
//   * the tile's histogram is kept in up to four LDS copies (lane l adds into
//     copy l mod copies) and summed in copy order;
//   * every tile writes its own partial row (S1, S2 compensated, histogram),
//     so the reduction kernel sums each integral's rows in tile order: the
//     result does not depend on which workgroup took which tile;
//   * the dimension and family are switched per tile to fully unrolled
//     instantiations (D = 1..12);
//   * begin (counter reset, a kernel, not a memset), persistent kernel,
//     reduction and refinement are captured once in a graph; per-iteration
//     inputs (iteration number, record slots) are read from device memory,
//     which the host updates before each replay;
//   * the tile size T and block size are chosen by timing candidate
//     configurations once per batch (autotuner), unless given.
#include "common.h"
#include "integrands.h"
#include "vegas_internal.h"

#include <algorithm>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

namespace vgx {

constexpr int BB_MAX = 256;  // launch bound of the persistent kernel
// Copies of a tile's LDS histogram (1, 2 or 4 per batch, as many as fit in
// kCopiesLds with the edges): lane l adds into copy l mod copies, so lanes of
// one atomic instruction that fall into the same bin mostly hit different
// addresses (LDS atomics on one address serialise); a copy is D nb + 1
// doubles so that a bin's copies fall on different banks.  The copies are
// summed in copy order when the tile's row is written.
constexpr int kMaxHistCopies = 4;
constexpr size_t kCopiesLds = 48 * 1024;
__host__ __device__ inline int hist_stride(int dim, int nb) { return dim * nb + 1; }
__host__ __device__ inline size_t batch_lds_bytes(int dim, int nb, int copies) {
  return sizeof(double) * ((size_t)dim * (nb + 1) + (size_t)copies * hist_stride(dim, nb));
}

struct BatchItem {
  int kind, prec, dim, nb;
  uint32_t sid, k0, k1;
  int pstride;           // 4 + dim * nb
  int64_t n;             // samples per iteration
  int64_t tile0;         // first tile of this integral
  int64_t ntiles;
  int64_t part_off;      // first double of this integral's tile partials
  double alpha;
  double* edges;         // context grid [dim][nb+1]
  double* hist;          // context histogram [dim][nb]
  IterRecord* rec;       // context records
  Combined* comb;
  IntegrandParams prm;
};

// Per-iteration inputs, one host-to-device copy: the tile counter, the
// iteration number, then the record slot of every integral (int32[count]).
struct BatchState {
  unsigned long long tile_counter;
  int iteration;
  int pad;
};
__host__ __device__ inline int* batch_krec(BatchState* st) { return (int*)(st + 1); }

template <int D, class F>
__device__ __forceinline__ void run_tile(const BatchItem& it, const F& f, const double* se, double* sh, int64_t s0,
                                         int64_t s1, uint32_t iter, Comp& c1, Comp& c2) {
  double p1 = 0.0, p2 = 0.0;
  // scaled coordinates t = u N straight from the Philox words (exact), the
  // Jacobian's constant N^D
  const double nbd = (double)it.nb, sc = nbd * 0x1p-32, hf = nbd * 0x1p-33;
  double nbD = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) nbD *= nbd;
  for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
    double t[D], x[D];
    int idx[D];
#pragma unroll
    for (int b = 0; b < (D + 3) / 4; ++b) {
      const u32x4 w4 = philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), iter, (it.sid << 8) | (uint32_t)b,
                                     it.k0, it.k1);
      const uint32_t ww[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (4 * b + e < D) t[4 * b + e < D ? 4 * b + e : 0] = fma((double)ww[e], sc, hf);
    }
    // edge pairs from global memory: the LDS holds the histogram copies
    const double jac = grid_map_t<D, true, true>(t, se, it.edges, it.nb, nbD, x, idx);
    const double w = f.eval(x) * jac;
    const double w2 = w * w;
    p1 += w;
    p2 += w2;
#pragma unroll
    for (int j = 0; j < D; ++j) atomicAdd(&sh[j * it.nb + idx[j]], w2);
  }
  c1.add(p1);
  c2.add(p2);
}

template <int D>
__device__ __forceinline__ void run_tile_d(const BatchItem& it, const double* se, double* sh, int64_t s0, int64_t s1,
                                           uint32_t iter, Comp& c1, Comp& c2) {
#define VGX_BT(T)                                                      \
  if (it.prec == VGX_F64) {                                            \
    T<D, double> f;                                                    \
    f.prm = it.prm;                                                    \
    run_tile<D>(it, f, se, sh, s0, s1, iter, c1, c2);                  \
  } else {                                                             \
    T<D, float> f;                                                     \
    f.prm = it.prm;                                                    \
    run_tile<D>(it, f, se, sh, s0, s1, iter, c1, c2);                  \
  }
  switch (it.kind) {
    case VGX_GAUSS: { VGX_BT(Gauss) break; }
    case VGX_GENZ_OSC: { VGX_BT(GenzOsc) break; }
    default: { VGX_BT(GenzPeak) break; }
  }
#undef VGX_BT
}

// Reset the tile counter at the start of an iteration (graph-safe: a kernel).
__global__ void k_batch_begin(BatchState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->tile_counter = 0ull;
}

__global__ __launch_bounds__(BB_MAX) void k_batch(const BatchItem* __restrict__ items, int count, int64_t total_tiles,
                                                 int tile, int copies, BatchState* __restrict__ st,
                                                 double* __restrict__ partials) {
  extern __shared__ double lds[];
  __shared__ int64_t s_tile;
  __shared__ int s_item;
  __shared__ double red[4][BB_MAX / 64];
  const uint32_t iter = (uint32_t)st->iteration;
  int cur = -1;
  double* se = lds;  // edges of the current integral [dim][nb+1]
  double* sh = nullptr;
  while (true) {
    if (threadIdx.x == 0) {
      const int64_t t = (int64_t)atomicAdd(&st->tile_counter, 1ull);
      s_tile = t;
      int lo = 0, hi = count - 1;  // integral owning tile t: last with tile0 <= t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile0 <= t) lo = mid; else hi = mid - 1;
      }
      s_item = lo;
    }
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= total_tiles) break;  // uniform: every wave leaves
    const int k = s_item;
    const BatchItem& it = items[k];
    const int ne = it.dim * (it.nb + 1);
    if (k != cur) {
      for (int q = threadIdx.x; q < ne; q += blockDim.x) se[q] = it.edges[q];
      cur = k;
    }
    sh = se + ne;
    const int hs = hist_stride(it.dim, it.nb);
    for (int q = threadIdx.x; q < copies * hs; q += blockDim.x) sh[q] = 0.0;
    __syncthreads();
    const int64_t lt = t - it.tile0;
    const int64_t s0 = lt * tile;
    const int64_t s1 = (s0 + tile < it.n) ? s0 + tile : it.n;
    Comp c1, c2;
    double* shl = sh + (threadIdx.x & (copies - 1)) * hs;  // this lane's histogram copy
    switch (it.dim) {
      case 1: run_tile_d<1>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 2: run_tile_d<2>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 3: run_tile_d<3>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 4: run_tile_d<4>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 5: run_tile_d<5>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 6: run_tile_d<6>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 7: run_tile_d<7>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 8: run_tile_d<8>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 9: run_tile_d<9>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 10: run_tile_d<10>(it, se, shl, s0, s1, iter, c1, c2); break;
      case 11: run_tile_d<11>(it, se, shl, s0, s1, iter, c1, c2); break;
      default: run_tile_d<12>(it, se, shl, s0, s1, iter, c1, c2); break;
    }
    const double v0 = wave_sum(c1.s), v1 = wave_sum(c1.c), v2 = wave_sum(c2.s), v3 = wave_sum(c2.c);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) { red[0][wv] = v0; red[1][wv] = v1; red[2][wv] = v2; red[3][wv] = v3; }
    __syncthreads();
    double* row = partials + it.part_off + lt * it.pstride;
    if (threadIdx.x < 4) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += red[threadIdx.x][q];
      row[threadIdx.x] = s;
    }
    for (int q = threadIdx.x; q < it.dim * it.nb; q += blockDim.x) {
      double h = sh[q];
      for (int c = 1; c < copies; ++c) h += sh[c * hs + q];
      row[4 + q] = h;
    }
    __syncthreads();  // LDS histogram and s_tile are reused by the next tile
  }
}

// Per integral (blockIdx.y) and column block (blockIdx.x): sum the tile rows
// in tile order; block x = 0 finalises the record and the combination, and
// copies the record to out[blockIdx.y] (all integrals' records in one array:
// one read-back).
__global__ __launch_bounds__(256) void k_batch_reduce(const BatchItem* __restrict__ items,
                                                      const double* __restrict__ partials, BatchState* st,
                                                      IterRecord* __restrict__ out) {
  const BatchItem& it = items[blockIdx.y];
  __shared__ double ss[4][64], sc[4][64];
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  const int ncols = it.pstride;
  if (blockIdx.x * 64 >= ncols) return;  // uniform per block
  Comp acc;
  if (col < ncols)
    for (int64_t r = grp; r < it.ntiles; r += 4) acc.add(partials[it.part_off + r * it.pstride + col]);
  ss[grp][lane] = acc.s;
  sc[grp][lane] = acc.c;
  __syncthreads();
  if (grp == 0) {
    Comp t;
    for (int g = 0; g < 4; ++g) { t.add(ss[g][lane]); t.add(sc[g][lane]); }
    ss[0][lane] = t.value();
    if (col >= 4 && col < ncols) it.hist[col - 4] = t.value();
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    const int k_rec = batch_krec(st)[blockIdx.y];
    finalize_record(ss[0][0] + ss[0][1], ss[0][2] + ss[0][3], it.n, it.rec, k_rec, it.comb);
    if (threadIdx.x == 0) out[blockIdx.y] = it.rec[k_rec];  // the lane that stored it
  }
}

// Per integral (blockIdx.y) and dimension (blockIdx.x): Lepage refinement.
__global__ __launch_bounds__(64) void k_batch_refine(const BatchItem* __restrict__ items, BatchState* st) {
  const BatchItem& it = items[blockIdx.y];
  if ((int)blockIdx.x >= it.dim) return;  // uniform per block
  refine_dim(it.edges + (size_t)blockIdx.x * (it.nb + 1), it.hist + (size_t)blockIdx.x * it.nb, it.nb, it.alpha);
}

}  // namespace vgx

using namespace vgx;

struct vgx_batch {
  int device = 0;
  hipStream_t stream = nullptr;      // replay stream (the first context's)
  hipStream_t cap = nullptr;         // private capture stream
  int count = 0;
  std::vector<vgx_vegas*> ctx;
  std::vector<int64_t> n;
  std::vector<BatchItem> items;      // host mirror
  BatchItem* d_items = nullptr;
  BatchState* d_state = nullptr;     // BatchState + int32 record slots [count]
  IterRecord* d_out = nullptr;       // this iteration's records [count]
  double* partials = nullptr;
  size_t part_cap = 0;               // doubles
  int tile = 0, block = 0, grid = 0;
  int copies = 1;                    // LDS histogram copies per workgroup
  int64_t total_tiles = 0;
  size_t lds = 0;
  int max_cols = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  IterRecord* pinned = nullptr;      // count records
  BatchState* pinned_state = nullptr;
};

namespace {

void layout(vgx_batch* b, int tile) {
  int64_t t0 = 0, off = 0;
  for (int k = 0; k < b->count; ++k) {
    BatchItem& it = b->items[k];
    it.tile0 = t0;
    it.ntiles = (b->n[k] + tile - 1) / tile;
    it.part_off = off;
    t0 += it.ntiles;
    off += it.ntiles * it.pstride;
  }
  b->total_tiles = t0;
  b->tile = tile;
}

size_t partial_doubles(const vgx_batch* b, int tile) {
  size_t off = 0;
  for (int k = 0; k < b->count; ++k) off += (size_t)((b->n[k] + tile - 1) / tile) * b->items[k].pstride;
  return off;
}

size_t state_bytes(int count) { return sizeof(BatchState) + sizeof(int) * (size_t)count; }

vgx_status upload_items(vgx_batch* b, hipStream_t st) {
  VGX_HIP(hipMemcpyAsync(b->d_items, b->items.data(), sizeof(BatchItem) * b->count, hipMemcpyHostToDevice, st));
  return VGX_OK;
}

vgx_status enqueue_iteration(vgx_batch* b, hipStream_t st, bool refine) {
  hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, st, b->d_state);
  hipLaunchKernelGGL(k_batch, dim3(b->grid), dim3(b->block), b->lds, st, b->d_items, b->count, b->total_tiles,
                     b->tile, b->copies, b->d_state, b->partials);
  if (refine) {
    hipLaunchKernelGGL(k_batch_reduce, dim3((b->max_cols + 63) / 64, b->count), dim3(256), 0, st, b->d_items,
                       b->partials, b->d_state, b->d_out);
    hipLaunchKernelGGL(k_batch_refine, dim3(VGX_MAX_DIM, b->count), dim3(64), 0, st, b->d_items, b->d_state);
  }
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

// Block size of the persistent kernel and a grid of as many workgroups as
// can be resident at once (the kernel's occupancy at that block size): more
// would only start once the tile queue is empty.
vgx_status set_block(vgx_batch* b, int block) {
  int per_cu = 0;
  VGX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_batch), block,
                                                       b->lds));
  b->block = block;
  b->grid = device_cus() * (per_cu > 0 ? per_cu : 1);
  return VGX_OK;
}

// Time the persistent kernel alone (grids untouched, records untouched) for
// candidate tile and block sizes; keep the fastest.
vgx_status autotune(vgx_batch* b, int fixed_tile, int fixed_block) {
  const int tiles[] = {2048, 4096, 8192, 16384, 32768};
  const int blocks[] = {128, 256};
  int best_t = fixed_tile > 0 ? fixed_tile : 8192, best_b = fixed_block > 0 ? fixed_block : 256;
  if (fixed_tile > 0 && fixed_block > 0) {
    layout(b, fixed_tile);
    return set_block(b, fixed_block);
  }
  hipEvent_t e0, e1;
  VGX_HIP(hipEventCreate(&e0));
  VGX_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  for (int ti : tiles) {
    if (fixed_tile > 0 && ti != fixed_tile) continue;
    for (int bl : blocks) {
      if (fixed_block > 0 && bl != fixed_block) continue;
      layout(b, ti);
      VGX_TRY(set_block(b, bl));
      VGX_TRY(upload_items(b, b->stream));
      float ms_best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        VGX_HIP(hipEventRecord(e0, b->stream));
        VGX_TRY(enqueue_iteration(b, b->stream, false));
        VGX_HIP(hipEventRecord(e1, b->stream));
        VGX_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        VGX_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms_best = ms < ms_best ? ms : ms_best;
      }
      if (ms_best < best) { best = ms_best; best_t = ti; best_b = bl; }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  layout(b, best_t);
  return set_block(b, best_b);
}

}  // namespace

extern "C" vgx_status batch_create(vgx_vegas* const* ctxs, int32_t count, const int64_t* n_samples, int32_t tile,
                                   int32_t block, void* stream, vgx_batch** out) {
  VGX_CHECK(out && ctxs && n_samples, "batch_create: null argument");
  *out = nullptr;
  VGX_CHECK(count >= 1 && count <= 65535, "batch_create: count out of 1..65535");
  VGX_CHECK(tile == 0 || (tile >= 256 && tile <= (1 << 24)), "batch_create: tile out of 256..2^24 (0 = autotune)");
  VGX_CHECK(block == 0 || block == 64 || block == 128 || block == 256, "batch_create: block must be 64/128/256 (0 = autotune)");
  int dev = 0;
  hipGetDevice(&dev);
  for (int k = 0; k < count; ++k) {
    VGX_CHECK(ctxs[k], "batch_create: null context %d", k);
    VGX_CHECK(ctxs[k]->kind != VGX_TTBAR && ctxs[k]->kind != VGX_DRELLYAN && ctxs[k]->kind != VGX_SINGLETOP,
              "batch_create: context %d has a PDF integrand (not batchable)", k);
    VGX_CHECK(ctxs[k]->device == dev, "batch_create: context %d is on another device", k);
    VGX_CHECK(n_samples[k] >= 2, "batch_create: n_samples[%d] < 2", k);
    for (int q = 0; q < k; ++q) VGX_CHECK(ctxs[q] != ctxs[k], "batch_create: context %d listed twice", k);
  }
  vgx_batch* b = new vgx_batch();
  b->device = dev;
  b->stream = stream ? (hipStream_t)stream : ctxs[0]->stream;
  b->count = count;
  b->ctx.assign(ctxs, ctxs + count);
  b->n.assign(n_samples, n_samples + count);
  b->items.resize(count);
  size_t max_lds[3] = {0, 0, 0};  // workgroup LDS with 1, 2, 4 histogram copies
  for (int k = 0; k < count; ++k) {
    const vgx_vegas* c = ctxs[k];
    BatchItem it{};
    it.kind = c->kind;
    it.prec = c->prec;
    it.dim = c->dim;
    it.nb = c->nb;
    it.sid = c->stream_id;
    it.k0 = (uint32_t)c->seed;
    it.k1 = (uint32_t)(c->seed >> 32);
    it.pstride = 4 + c->dim * c->nb;
    it.n = n_samples[k];
    it.alpha = c->alpha;
    it.edges = c->edges;
    it.hist = c->hist;
    it.rec = c->rec;
    it.comb = c->comb;
    it.prm = c->prm;
    b->items[k] = it;
    for (int q = 0; q < 3; ++q) max_lds[q] = std::max(max_lds[q], batch_lds_bytes(c->dim, c->nb, 1 << q));
    b->max_cols = it.pstride > b->max_cols ? it.pstride : b->max_cols;
  }
  b->copies = max_lds[2] <= kCopiesLds ? 4 : (max_lds[1] <= kCopiesLds ? 2 : 1);
  b->lds = max_lds[b->copies == 4 ? 2 : b->copies - 1];
  vgx_status s = VGX_OK;
  do {
    b->part_cap = partial_doubles(b, tile > 0 ? tile : 2048);
    if ((s = dev_alloc((void**)&b->partials, sizeof(double) * b->part_cap)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&b->d_items, sizeof(BatchItem) * count)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&b->d_state, state_bytes(count))) != VGX_OK) break;
    if ((s = dev_alloc((void**)&b->d_out, sizeof(IterRecord) * count)) != VGX_OK) break;
    if ((s = host_alloc((void**)&b->pinned, sizeof(IterRecord) * count)) != VGX_OK) break;
    if ((s = host_alloc((void**)&b->pinned_state, state_bytes(count))) != VGX_OK) break;
  } while (0);
  if (s != VGX_OK) { batch_destroy(b); return s; }
  hipError_t e = hipMemsetAsync(b->d_state, 0, state_bytes(count), b->stream);
  if (e != hipSuccess) { s = hip_fail(e, "batch_create", __FILE__, __LINE__); batch_destroy(b); return s; }
  s = autotune(b, tile, block);
  if (s == VGX_OK) s = upload_items(b, b->stream);
  if (s == VGX_OK) {
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) s = hip_fail(e, "batch_create autotune", __FILE__, __LINE__);
  }
  // capture one iteration into a graph on a private stream
  if (s == VGX_OK) {
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      vgx_status cs = enqueue_iteration(b, b->cap, true);
      hipError_t e2 = hipStreamEndCapture(b->cap, &b->graph);
      if (cs != VGX_OK) s = cs;
      else if (e2 != hipSuccess) e = e2;
    }
    if (s == VGX_OK && e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (s == VGX_OK && e != hipSuccess) s = hip_fail(e, "batch_create graph capture", __FILE__, __LINE__);
  }
  if (s != VGX_OK) { batch_destroy(b); return s; }
  *out = b;
  return VGX_OK;
}

extern "C" vgx_status batch_iterate(vgx_batch* b, int32_t iteration, vgx_iter_result* out) {
  VGX_CHECK(b, "batch_iterate: null batch");
  // per-iteration inputs in one copy: the iteration number and each
  // integral's record slot (its context's count of stored records)
  int* krec = batch_krec(b->pinned_state);
  for (int k = 0; k < b->count; ++k) {
    if (b->ctx[k]->n_rec >= MAX_RECORDS) { set_error("batch_iterate: context %d has too many records", k); return VGX_ESTATE; }
    if (b->ctx[k]->pend_k >= 0) {  // a record left pending on the context's own stream
      VGX_TRY(vegas_flush_pending(b->ctx[k]));
      VGX_HIP(hipStreamSynchronize(b->ctx[k]->stream));
    }
    krec[k] = b->ctx[k]->n_rec;
  }
  b->pinned_state->tile_counter = 0;
  b->pinned_state->iteration = iteration;
  b->pinned_state->pad = 0;
  VGX_HIP(hipMemcpyAsync(b->d_state, b->pinned_state, state_bytes(b->count), hipMemcpyHostToDevice, b->stream));
  VGX_HIP(hipGraphLaunch(b->exec, b->stream));
  VGX_HIP(hipMemcpyAsync(b->pinned, b->d_out, sizeof(IterRecord) * b->count, hipMemcpyDeviceToHost, b->stream));
  VGX_HIP(hipStreamSynchronize(b->stream));
  vgx_status s = VGX_OK;
  for (int k = 0; k < b->count; ++k) {
    b->ctx[k]->n_rec++;
    b->ctx[k]->comb_fresh = false;
    b->ctx[k]->have_hist = true;
    const IterRecord& r = b->pinned[k];
    if (out) {
      out[k].mean = r.mean;
      out[k].var = r.var;
      out[k].s1 = r.s1;
      out[k].s2 = r.s2;
      out[k].n = r.n;
    }
    if (!r.finite && s == VGX_OK) {
      set_error("batch_iterate: integral %d gave a non-finite estimate (excluded)", k);
      s = VGX_ENUMERIC;
    }
  }
  return s;
}

extern "C" vgx_status batch_config(vgx_batch* b, int32_t* tile, int32_t* block) {
  VGX_CHECK(b && tile && block, "batch_config: null argument");
  *tile = b->tile;
  *block = b->block;
  return VGX_OK;
}

extern "C" void batch_destroy(vgx_batch* b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap) hipStreamDestroy(b->cap);
  hipFree(b->partials);
  hipFree(b->d_items);
  hipFree(b->d_state);
  hipFree(b->d_out);
  if (b->pinned) hipHostFree(b->pinned);
  if (b->pinned_state) hipHostFree(b->pinned_state);
  delete b;
}
