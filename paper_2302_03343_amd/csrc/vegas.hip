// VEGAS adaptive importance sampling on the GPU: Philox uniforms -> grid map
// with Jacobian -> fused integrand -> compensated sums and per-bin
// histograms -> fixed-order reduction -> estimate and combination -> grid
// refinement.
//
// Thesis: importance-sampling estimator E_N = (1/N) sum f/p and its variance
// (MC chapter, importance-sampling equations); VEGAS (Sec. "Adaptive Monte
// Carlo: VEGAS algorithm"): separable grid, fixed bin count, adaptive
// widths, inverse-variance combination of iterations and the chi^2/dof
// check; sampling by the inverse-transform method (Sec. "Inverse transform
// method").  The refinement (smoothing, damping, re-binning) is Lepage's
// (1978), which the thesis cites but does not print.
//
// MI355X design
//   * one fused kernel per iteration, grid-stride over the sample indices
//     (32-bit within segments whose counters do not carry), no per-sample
//     buffers: uniforms are regenerated from the counter;
//   * the grid edges (d x (N+1) FP64) and the per-workgroup histogram
//     (d x N FP64, LDS atomics) live in LDS; integrand tables (the PDF rows
//     of the hadronic integrands) too, staged once per context and copied
//     by every workgroup;
//   * S1, S2 are FP64 sums compensated per 16-sample chunk (Neumaier), wave
//     reduced with cross-lane shuffles and written as per-workgroup partials;
//     a second kernel reduces the partials in a fixed order (no float
//     atomics across workgroups), computes E and var(E), and updates the
//     inverse-variance combination, all on the device;
//   * refinement runs as one workgroup per dimension.
#include "common.h"
#include "integrands.h"
#include "pdf_internal.h"
#include "ttbar.h"
#include "drellyan.h"
#include "singletop.h"
#include "ttbar_dyn.h"
#include "vegas_internal.h"
#include "flow_internal.h"

#include <math.h>
#include <stdlib.h>

#include <type_traits>

namespace vgx {

constexpr int BLOCK = 256;
constexpr int CHUNK = 16;

struct VegasArgs {
  int64_t n;
  const double* edges;
  int nb;
  int pstride;   // doubles per workgroup partial row
  int hcopies;   // histogram copies in LDS: 4 per wave, one per wave, or 1 (shared)
  double nbD;    // nb^dim, the Jacobian's constant factor
  double sc;     // nb 2^-32: t = u nb = (word + 1/2) sc
  // the integrand's LDS tables as staged once for the context (copied by
  // each workgroup), or null (each workgroup stages them itself)
  const float* tables;
  int table_bytes;  // a multiple of 16
};

// Histogram copies a workgroup keeps in LDS: one per wave when they fit in
// 16 KB (each wave's atomics then meet only its own lanes, and the copies are
// summed in wave order), else one shared by all waves.  Integrands that stage
// no tables in LDS (lane_groups) take four per wave when they fit in 32 KB,
// lane l of wave w adding into copy 4 w + l mod 4: lanes of one atomic
// instruction that fall into the same bin then mostly hit different
// addresses (LDS atomics on one address serialise).
__host__ __device__ inline int hist_copies(int D, int nb, bool lane_groups) {
  const int waves = BLOCK / 64, bytes = D * nb * (int)sizeof(double);
  if (lane_groups && 4 * waves * bytes <= 32768) return 4 * waves;
  return waves * bytes <= 16384 ? waves : 1;
}

// ---------------------------------------------------------------------------
// Sample sources
// ---------------------------------------------------------------------------
template <int D>
struct PhiloxSrc {
  static constexpr bool kInterior = true;  // 0 < u N < N for every sample
  uint32_t it, sid, k0, k1;
  int64_t first;
  __device__ __forceinline__ double get(int64_t i, double (&u)[D]) const {
    philox_uniforms<D>((uint64_t)(first + i), it, sid, k0, k1, u);
    return 1.0;
  }
  // scaled coordinates t = u N = (k + 1/2) N 2^-32 of counter (c0, c1), exact
  // (k N 2^-32 has at most 40 significant bits): one FMA with the two
  // constants in registers, or (LEAN, for register-bound kernels) k + 1/2
  // (an inline constant) times the uniform scale, two instructions and no
  // vector registers for the constants
  template <bool LEAN>
  __device__ __forceinline__ double get_t_c(uint32_t c0, uint32_t c1, double sc, double hf, double (&t)[D]) const {
#pragma unroll
    for (int b = 0; b < (D + 3) / 4; ++b) {
      const u32x4 w = philox4x32_10(c0, c1, it, (sid << 8) | (uint32_t)b, k0, k1);
      const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (4 * b + e < D)
          t[4 * b + e < D ? 4 * b + e : 0] = LEAN ? ((double)ww[e] + 0.5) * sc : fma((double)ww[e], sc, hf);
    }
    return 1.0;
  }
  // Samples are taken in segments within which the low counter word does
  // not carry: 32-bit indices i, counter (first + base) + i, at most 2^31
  // per segment (so that i + grid stride cannot wrap either).
  __host__ __device__ __forceinline__ int64_t seg_len(int64_t base, int64_t left) const {
    const int64_t room = ((int64_t)1 << 31) - (int64_t)((uint64_t)(first + base) & 0x7FFFFFFFu);
    return left < room ? left : room;
  }
  template <bool LEAN>
  __device__ __forceinline__ double get_t_seg(int64_t base, uint32_t i, double nbd, double sc, double hf,
                                              double (&t)[D]) const {
    const uint64_t c = (uint64_t)(first + base);
    return get_t_c<LEAN>((uint32_t)c + i, (uint32_t)(c >> 32), sc, hf, t);
  }
};

template <int D>
struct PointsSrc {
  static constexpr bool kInterior = false;  // caller points may lie on the faces
  const double* y;     // [D][n]
  const double* logq;  // [n] or null
  int64_t n;
  __device__ __forceinline__ double get(int64_t i, double (&u)[D]) const {
#pragma unroll
    for (int j = 0; j < D; ++j) u[j] = y[(int64_t)j * n + i];
    return logq ? exp(-logq[i]) : 1.0;
  }
  __host__ __device__ __forceinline__ int64_t seg_len(int64_t base, int64_t left) const {
    return left < ((int64_t)1 << 31) ? left : ((int64_t)1 << 31);
  }
  template <bool LEAN>
  __device__ __forceinline__ double get_t_seg(int64_t base, uint32_t i32, double nbd, double sc, double hf,
                                              double (&t)[D]) const {
    const int64_t i = base + i32;
#pragma unroll
    for (int j = 0; j < D; ++j) t[j] = y[(int64_t)j * n + i] * nbd;
    return logq ? exp(-logq[i]) : 1.0;
  }
};

// Offset (in doubles, even: 16-byte aligned) of the integrand tables after
// the edges [D][nb+1] and, with histograms, [copies][D][nb].
__host__ __device__ inline int lds_table_offset(int D, int nb, bool hist, bool lane_groups) {
  const int n = D * (nb + 1) + (hist ? hist_copies(D, nb, lane_groups) * D * nb : 0);
  return (n + 1) & ~1;
}

// ---------------------------------------------------------------------------
// Integrand tables in LDS.  An integrand that stages tables (PDF rows, knots,
// per-cell Hermite inputs) computes them from the PDF grid with scattered
// loads and index arithmetic; k_stage_tables does that once per context, in
// one workgroup, and stores the LDS block as it stands, so that each
// workgroup of a launch only copies it (16-byte loads, all in flight): the
// same LDS contents, bit for bit.
// ---------------------------------------------------------------------------
template <class F>
__global__ __launch_bounds__(BLOCK) void k_stage_tables(F f, float* __restrict__ out, int bytes) {
  extern __shared__ __align__(16) float tl[];
  F ff = f;
  ff.stage(tl);
  __syncthreads();
  copy16(out, tl, bytes);
}

template <class F>
__device__ __forceinline__ void stage_tables(F& ff, float* extra, const VegasArgs& a) {
  if (a.tables) {
    ff.layout(extra);
    copy16(extra, a.tables, a.table_bytes);
  } else {
    ff.stage(extra);
  }
}

// ---------------------------------------------------------------------------
// Fused iteration kernel.
// LDS: edges [D][nb+1] | histogram [D][nb] (HIST) | integrand staging.
// Partial row per workgroup: [S1.s, S1.c, S2.s, S2.c, hist[D][nb]].
// ---------------------------------------------------------------------------
// Minimum waves per SIMD an integrand asks of the iteration kernel (its
// register budget): F::kMinWaves when declared, else 1 (no constraint).
template <class F, class = void>
struct MinWaves { static constexpr int value = 1; };
template <class F>
struct MinWaves<F, std::void_t<decltype(F::kMinWaves)>> { static constexpr int value = F::kMinWaves; };

// Caller points (flow samples) carry a density and an index into memory:
// the integrand's occupancy bound would make those kernels spill, so they
// take none.
template <int D, class F, class Src, bool HIST, bool WIDE = false>
__global__ __launch_bounds__(BLOCK, Src::kInterior ? MinWaves<F>::value : 1) void k_vegas_iter(VegasArgs a, F f, Src src,
                                                                          double* __restrict__ partials) {
  extern __shared__ __align__(16) double lds[];
  const int nb = a.nb;
  double* se = lds;
  double* sh = se + D * (nb + 1);
  // integrand tables start on a 16-byte boundary (they are read as float4)
  float* extra = (float*)(lds + lds_table_offset(D, nb, HIST, !F::kStage));
  for (int k = threadIdx.x; k < D * (nb + 1); k += BLOCK) se[k] = a.edges[k];
  if (HIST)
    for (int k = threadIdx.x; k < a.hcopies * D * nb; k += BLOCK) sh[k] = 0.0;
  F ff = f;
  if constexpr (F::kStage) stage_tables(ff, extra, a);
  __syncthreads();
  // The epilogue rebuilds the thread index from the wave index (uniform, so
  // a scalar register) and the lane (mbcnt), so that no vector register has
  // to carry it across the sample loop.
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // this wave's (integrands with LDS tables: a uniform pointer) or this
  // lane's histogram copy
  double* hw;
  if constexpr (F::kStage) {
    hw = sh + (a.hcopies > 1 ? wv * D * nb : 0);
  } else {
    const int hc = a.hcopies > BLOCK / 64 ? 4 * wv + (int)(threadIdx.x & 3) : (a.hcopies > 1 ? wv : 0);
    hw = sh + hc * D * nb;
  }

  Comp c1, c2;
  double p1 = 0.0, p2 = 0.0;
  const double nbd = (double)nb, sc = a.sc, hf = nbd * 0x1p-33;
  // one sample from its scaled coordinates and source weight
  auto sample = [&](const double (&t)[D], double ws) {
    double x[D];
    int idx[D];
    // integrands without LDS tables: the edge pairs come from global memory
    const double jac = grid_map_t<D, Src::kInterior, !F::kStage>(t, se, a.edges, nb, a.nbD, x, idx);
    const double w = ff.eval(x) * jac * ws;
    const double w2 = w * w;
    p1 += w;
    p2 += w2;
    if (HIST) {
#pragma unroll
      for (int j = 0; j < D; ++j) atomicAdd(&hw[j * nb + idx[j]], w2);
    }
  };
  // 32-bit sample indices: no 64-bit adds and compares in the loop.  WIDE
  // launches (the low counter word would carry, or more than 2^31 samples)
  // run in segments that do not; each thread adds CHUNK of its samples into
  // the compensated sums at a time.
  const uint32_t stride = gridDim.x * BLOCK;
  int cnt = 0;
  auto run = [&](int64_t base, uint32_t len) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < len; i += stride) {
      double t[D];
      // integrands with LDS tables are register-bound (occupancy)
      const double ws = src.template get_t_seg<F::kStage>(base, i, nbd, sc, hf, t);
      sample(t, ws);
      if (++cnt == CHUNK) {
        c1.add(p1);
        c2.add(p2);
        p1 = p2 = 0.0;
        cnt = 0;
      }
    }
  };
  if constexpr (WIDE) {
    for (int64_t base = 0; base < a.n;) {
      const uint32_t len = (uint32_t)src.seg_len(base, a.n - base);
      run(base, len);
      base += len;
    }
  } else {
    run(0, (uint32_t)a.n);
  }
  c1.add(p1);
  c2.add(p2);

  __shared__ double red[4][BLOCK / 64];
  const double v0 = wave_sum(c1.s), v1 = wave_sum(c1.c), v2 = wave_sum(c2.s), v3 = wave_sum(c2.c);
  const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const int tid = wv * 64 + lane;
  if (lane == 0) { red[0][wv] = v0; red[1][wv] = v1; red[2][wv] = v2; red[3][wv] = v3; }
  __syncthreads();
  double* row = partials + (size_t)blockIdx.x * a.pstride;
  if (tid < 4) {
    double s = 0.0;
    for (int k = 0; k < BLOCK / 64; ++k) s += red[tid][k];
    row[tid] = s;
  }
  if (HIST)
    for (int k = tid; k < D * nb; k += BLOCK) {
      double h = sh[k];
      for (int c = 1; c < a.hcopies; ++c) h += sh[c * D * nb + k];  // copy order
      row[4 + k] = h;
    }
}

// ---------------------------------------------------------------------------
// Fused flow-sampling iteration: the importance-sampling estimate with the
// coupling flow as the proposal density q.  Each wave draws a 64-sample tile
// pair from the flow as flow_sample draws it (Philox u, the coupling layers
// in the sampling direction: y and log q in the lane of each sample), maps
// y through the VEGAS grid and weights f(x) J(y) / q(y) into compensated S1
// and S2, as the iteration kernel does with caller points and their log q;
// nothing per sample goes to HBM.  LDS: edges [D][nb+1] | integrand tables |
// flow packs | biases | per-lane columns [d][FI_BLOCK].
// ---------------------------------------------------------------------------
struct FlowIterArgs {
  const FlowDesc* desc;
  const void* fw;
  const float* bias;
  int flow_off;  // byte offset of the flow's part of the LDS (16-byte aligned)
  uint32_t it, sid, k0, k1;
};

constexpr int FI_BLOCK = 512;  // eight waves share one LDS copy of the weights and tables

template <int D, class F, class OP>
__global__ __launch_bounds__(FI_BLOCK) void k_flow_iter(VegasArgs a, F f, FlowIterArgs fa,
                                                        double* __restrict__ partials) {
  using S = typename OP::S;
  extern __shared__ __align__(16) double lds[];
  const int nb = a.nb;
  double* se = lds;
  float* extra = (float*)(lds + lds_table_offset(D, nb, false, !F::kStage));
  unsigned char* fl = (unsigned char*)lds + fa.flow_off;
  const FlowDesc& FD = *fa.desc;
  S* sfw = (S*)fl;
  float* sb = (float*)(fl + (size_t)FD.fw_total * sizeof(S));
  float* z = (float*)(fl + fwd_z_offset(FD.fw_total, FD.bias_total, (int)sizeof(S))) + threadIdx.x;
  for (int k = threadIdx.x; k < D * (nb + 1); k += FI_BLOCK) se[k] = a.edges[k];
  F ff = f;
  if constexpr (F::kStage) stage_tables(ff, extra, a);
  copy16(sfw, fa.fw, FD.fw_total * (int)sizeof(S));
  copy16(sb, fa.bias, FD.bias_total * 4);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = (threadIdx.x >> 6) * gridDim.x + blockIdx.x;
  const int nwaves = gridDim.x * (FI_BLOCK / 64);
  const int64_t npairs = (a.n + 63) / 64;
  const double nbd = (double)nb;
  Comp c1, c2;
  double p1 = 0.0, p2 = 0.0;
  int cnt = 0;
  for (int64_t t = wave; t < npairs; t += nwaves) {
    const int64_t i = t * 64 + lane;  // the lane's own sample; every lane runs the layers
    const bool valid = i < a.n;
    flow_draw<FI_BLOCK>(z, D, i, fa.it, fa.sid, fa.k0, fa.k1);
    const double lq = flow_layers<true, OP, FI_BLOCK>(FD, sfw, sb, z, i, valid, nullptr, a.n);
    if (valid) {
      double tt[D], x[D];
      int idx[D];
#pragma unroll
      for (int j = 0; j < D; ++j) tt[j] = (double)z[j * FI_BLOCK] * nbd;
      const double jac = grid_map_t<D, false, !F::kStage>(tt, se, a.edges, nb, a.nbD, x, idx);
      const double w = ff.eval(x) * jac * exp(-lq);
      p1 += w;
      p2 += w * w;
      if (++cnt == CHUNK) {
        c1.add(p1);
        c2.add(p2);
        p1 = p2 = 0.0;
        cnt = 0;
      }
    }
  }
  c1.add(p1);
  c2.add(p2);
  __shared__ double red[4][FI_BLOCK / 64];
  const double v0 = wave_sum(c1.s), v1 = wave_sum(c1.c), v2 = wave_sum(c2.s), v3 = wave_sum(c2.c);
  const int wv = threadIdx.x >> 6;
  if (lane == 0) { red[0][wv] = v0; red[1][wv] = v1; red[2][wv] = v2; red[3][wv] = v3; }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int k = 0; k < FI_BLOCK / 64; ++k) s += red[threadIdx.x][k];
    partials[(size_t)blockIdx.x * a.pstride + threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the partial rows.  Workgroup b owns the 8 columns
// 8b .. 8b+7.  Thread (g, c) of its 128 row groups sums rows g, g+128, ...
// of column c with compensation, after issuing all of its loads (at most
// RMAXR); the groups are then merged in a fixed order: across the 8 groups
// of a wave by shuffles, then across the 16 waves through LDS.  Workgroup 0
// (which owns S1 and S2) turns (S1, S2, n) into the iteration record and
// updates the combination, or, with defer set, stores only S1 and S2 in the
// record: the record is then completed by the next refinement, in a
// workgroup of its own beside the dimensions' workgroups, or by k_finalize.
// ---------------------------------------------------------------------------
constexpr int RBLOCK = 1024;
constexpr int RCOLS = 8;
constexpr int RGROUPS = RBLOCK / RCOLS;
constexpr int RMAXR = 16;
constexpr int RMAXROWS = RGROUPS * RMAXR;

__global__ __launch_bounds__(RBLOCK) void k_reduce(const double* __restrict__ partials, int rows, int pstride,
                                                   int ncols, double* __restrict__ hist_out, int64_t n,
                                                   IterRecord* __restrict__ rec, int k_rec, Combined* __restrict__ comb,
                                                   int defer) {
  __shared__ double ss[RBLOCK / 64][RCOLS], sc[RBLOCK / 64][RCOLS];
  __shared__ double tot[RCOLS];
  const int cl = threadIdx.x % RCOLS, grp = threadIdx.x / RCOLS;
  const int col = blockIdx.x * RCOLS + cl;
  Comp acc;
  if (col < ncols) {
    double v[RMAXR];
#pragma unroll
    for (int q = 0; q < RMAXR; ++q) {
      const int r = grp + q * RGROUPS;
      v[q] = r < rows ? partials[(size_t)r * pstride + col] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < RMAXR; ++q)
      if (grp + q * RGROUPS < rows) acc.add(v[q]);
  }
  // lanes l and l^8, l^16, l^32 hold the same column
#pragma unroll
  for (int m = RCOLS; m < 64; m <<= 1) {
    const double os = __shfl_xor(acc.s, m, 64), oc = __shfl_xor(acc.c, m, 64);
    acc.add(os);
    acc.c += oc;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane < RCOLS) {
    ss[wv][lane] = acc.s;
    sc[wv][lane] = acc.c;
  }
  __syncthreads();
  if (threadIdx.x < RCOLS) {
    Comp t;
    t.s = ss[0][cl];
    t.c = sc[0][cl];
    for (int k = 1; k < RBLOCK / 64; ++k) {
      t.add(ss[k][cl]);
      t.c += sc[k][cl];
    }
    const double v = t.value();
    tot[cl] = v;
    if (col >= 4 && col < ncols) hist_out[col - 4] = v;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    if (!defer) {
      finalize_record(tot[0] + tot[1], tot[2] + tot[3], n, rec, k_rec, comb);
    } else if (threadIdx.x == 0) {
      rec[k_rec].s1 = tot[0] + tot[1];
      rec[k_rec].s2 = tot[2] + tot[3];
    }
  }
}

// Refinement, one workgroup per dimension; with k_pend >= 0 the grid has one
// more workgroup, which completes the deferred record k_pend of n_pend
// samples from the S1 and S2 stored in it (the refinement does not read it).
__global__ __launch_bounds__(64) void k_refine(double* __restrict__ edges, const double* __restrict__ hist, int nb,
                                               double alpha, IterRecord* __restrict__ rec, int k_pend, int64_t n_pend,
                                               Combined* __restrict__ comb) {
  if (k_pend >= 0 && blockIdx.x == gridDim.x - 1) {
    finalize_record(rec[k_pend].s1, rec[k_pend].s2, n_pend, rec, k_pend, comb);
    return;
  }
  refine_dim(edges + (size_t)blockIdx.x * (nb + 1), hist + (size_t)blockIdx.x * nb, nb, alpha);
}

__global__ __launch_bounds__(64) void k_finalize(IterRecord* __restrict__ rec, int k, int64_t n,
                                                 Combined* __restrict__ comb) {
  finalize_record(rec[k].s1, rec[k].s2, n, rec, k, comb);
}

// ---------------------------------------------------------------------------
// Materialise samples: u [D][n] and g = f(G(u)) J(u).
// ---------------------------------------------------------------------------
template <int D, class F>
__global__ __launch_bounds__(BLOCK) void k_vegas_sample(VegasArgs a, F f, PhiloxSrc<D> src, double* __restrict__ u_out,
                                                        double* __restrict__ g_out) {
  extern __shared__ __align__(16) double lds[];
  const int nb = a.nb;
  double* se = lds;
  float* extra = (float*)(lds + lds_table_offset(D, nb, false, !F::kStage));
  for (int k = threadIdx.x; k < D * (nb + 1); k += BLOCK) se[k] = a.edges[k];
  F ff = f;
  if constexpr (F::kStage) stage_tables(ff, extra, a);
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < a.n; i += stride) {
    double u[D], x[D];
    int idx[D];
    src.get(i, u);
    const double jac = grid_map<D>(u, se, nb, x, idx);
    if (u_out) {
#pragma unroll
      for (int j = 0; j < D; ++j) u_out[(int64_t)j * a.n + i] = u[j];
    }
    if (g_out) g_out[i] = ff.eval(x) * jac;
  }
}

}  // namespace vgx

using namespace vgx;

namespace {

bool uses_pdf(int kind) { return kind == VGX_TTBAR || kind == VGX_DRELLYAN || kind == VGX_SINGLETOP; }

// Bytes of the integrand's LDS tables, a multiple of 16 (they are copied in
// 16-byte pieces).
size_t extra_lds_bytes(const vgx_vegas* v) {
  size_t floats = 0;
  if (v->kind == VGX_TTBAR && v->tt_dyn) floats = (size_t)ttdyn_lds_floats(v->ttd.nxs, v->ttd.R, v->ttd.a_nq);
  else if (v->kind == VGX_TTBAR) floats = (size_t)pdf_rows_lds_floats(v->tt.pdf.nxs);
  else if (v->kind == VGX_DRELLYAN) floats = (size_t)pdf_rows_lds_floats(v->dy.pdf.nxs);
  else if (v->kind == VGX_SINGLETOP) floats = (size_t)pdf_rows_lds_floats(v->st.pdf.nxs);
  return (sizeof(float) * floats + 15) & ~(size_t)15;
}

// Resident workgroups per CU of a hadronic integrand's iteration kernel (its
// LDS footprint and registers decide); one grid-stride wave of workgroups
// fills the chip.
int hadronic_blocks_per_cu(const vgx_vegas* v) {
  int occ = 0;
  const size_t lds = sizeof(double) * (size_t)lds_table_offset(3, v->nb, true, false) + extra_lds_bytes(v);
  const void* k = (v->kind == VGX_TTBAR && v->tt_dyn)
                      ? reinterpret_cast<const void*>(&k_vegas_iter<3, TTbarDyn, PhiloxSrc<3>, true>)
                  : v->kind == VGX_TTBAR    ? reinterpret_cast<const void*>(&k_vegas_iter<3, TTbar, PhiloxSrc<3>, true>)
                  : v->kind == VGX_DRELLYAN ? reinterpret_cast<const void*>(&k_vegas_iter<3, DrellYan, PhiloxSrc<3>, true>)
                                            : reinterpret_cast<const void*>(&k_vegas_iter<3, SingleTop, PhiloxSrc<3>, true>);
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, BLOCK, lds);
  if (e != hipSuccess || occ < 1) {
    (void)hipGetLastError();
    occ = 4;
  }
  return occ > 8 ? 8 : occ;
}

template <class F>
vgx_status stage_tables_once(vgx_vegas* v, const F& f) {
  const int bytes = v->table_bytes;
  if (bytes > 65536)
    VGX_HIP(hipFuncSetAttribute((const void*)k_stage_tables<F>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  hipLaunchKernelGGL((k_stage_tables<F>), dim3(1), dim3(BLOCK), (size_t)bytes, v->stream, f, v->tables, bytes);
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

// The hadronic integrands' LDS tables, staged once into v->tables.
vgx_status build_tables(vgx_vegas* v) {
  if (!uses_pdf(v->kind)) return VGX_OK;
  v->table_bytes = (int)extra_lds_bytes(v);
  VGX_TRY(dev_alloc((void**)&v->tables, (size_t)v->table_bytes));
  if (v->kind == VGX_TTBAR && v->tt_dyn) {
    TTbarDyn f{};
    f.c = v->ttd;
    return stage_tables_once(v, f);
  }
  if (v->kind == VGX_TTBAR) {
    TTbar f{};
    f.c = v->tt;
    return stage_tables_once(v, f);
  }
  if (v->kind == VGX_DRELLYAN) {
    DrellYan f{};
    f.c = v->dy;
    return stage_tables_once(v, f);
  }
  SingleTop f{};
  f.c = v->st;
  return stage_tables_once(v, f);
}

int grid_for(const vgx_vegas* v, int64_t n) {
  const int64_t want = (n + BLOCK - 1) / BLOCK;
  return (int)(want < v->max_wg ? (want > 0 ? want : 1) : v->max_wg);
}

// Cell-guess constants for knots v[0..n) uniform in their logarithm to 1e-3
// of a spacing: first logarithm and inverse spacing; false when not uniform
// (the kernels then search).
bool uniform_log_knots(const double* v, int n, float& l0f, float& inv_d) {
  const double l0 = log(v[0]), d = (log(v[n - 1]) - l0) / (n - 1);
  bool uni = true;
  for (int k = 0; k < n; ++k)
    if (fabs(log(v[k]) - (l0 + k * d)) > 1e-3 * d) uni = false;
  l0f = (float)l0;
  inv_d = (float)(1.0 / d);
  return uni;
}

// PDF rows at the fixed scale mu2 for an integrand whose momentum fractions
// never fall below x_min.
vgx_status setup_pdf_rows(PdfRowsConst& t, const vgx_pdf* pdf, double mu2, double x_min, bool contract,
                          const char* who) {
  VGX_CHECK(pdf->n_flav == TT_NF, "%s needs an 11-flavour PDF (order -5..-1, g, 1..5)", who);
  VGX_CHECK(pdf->n_x <= TT_MAX_NX, "%s supports at most %d x knots", who, TT_MAX_NX);
  VGX_CHECK(x_min >= pdf->h_x[0], "%s: smallest momentum fraction below the PDF x range", who);
  int sub = -1;
  for (int k = 0; k < pdf->n_sub; ++k) {
    const double lo = pdf->h_q2[pdf->q_off[k]], hi = pdf->h_q2[pdf->q_off[k] + pdf->nq[k] - 1];
    const bool last = k == pdf->n_sub - 1;
    if (mu2 >= lo && (mu2 < hi || (last && mu2 <= hi))) sub = k;
  }
  VGX_CHECK(sub >= 0, "%s: mu^2 outside the PDF Q^2 range", who);
  const double* q = pdf->h_q2 + pdf->q_off[sub];
  const int nq = pdf->nq[sub];
  int j = 0;
  while (j < nq - 2 && q[j + 1] <= mu2) ++j;
  t.v32 = pdf->v32;
  t.fstride = pdf->fstride;
  t.lx = pdf->lx;
  t.n_x = pdf->n_x;
  // every event has ln x >= ln x_min; stage from two cells below the cell of
  // x_min (margin for FP32 rounding of ln x)
  int i0 = 0;
  while (i0 < pdf->n_x - 2 && pdf->h_x[i0 + 1] <= x_min) ++i0;
  t.ix0 = i0 >= 2 ? i0 - 2 : 0;
  if (pdf->n_x - t.ix0 < 4) t.ix0 = pdf->n_x - 4 > 0 ? pdf->n_x - 4 : 0;
  t.nxs = pdf->n_x - t.ix0;
  VGX_CHECK(t.nxs >= 4, "%s needs at least 4 x knots", who);
  if (j >= 1 && j <= nq - 3) { t.n_rows = 4; t.row0 = pdf->q_off[sub] + j - 1; }
  else { t.n_rows = 2; t.row0 = pdf->q_off[sub] + j; }
  t.contract = contract ? 1 : 0;
  // Q-row weights at mu^2 (FP64, stored FP32): the cubic Hermite with secant
  // slopes on the four rows around mu^2, linear on the cell when two rows are
  // staged; ql: linear on the cell (j, j + 1), rows 1, 2 of four or 0, 1 of two
  {
    const double lj = log(q[j]), lj1 = log(q[j + 1]);
    const double hb = lj1 - lj;
    const double tb = (log(mu2) - lj) / hb;
    if (t.n_rows == 4) {
      const double rm = hb / (lj - log(q[j - 1])), rp = hb / (log(q[j + 2]) - lj1);
      const double t2 = tb * tb, t3 = t2 * tb;
      const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + tb, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
      t.qh[0] = (float)(-0.5 * h10 * rm);
      t.qh[1] = (float)(h00 - 0.5 * h10 + 0.5 * h10 * rm - 0.5 * h11);
      t.qh[2] = (float)(h01 + 0.5 * h10 - 0.5 * h11 * rp + 0.5 * h11);
      t.qh[3] = (float)(0.5 * h11 * rp);
      t.ql[0] = 0.0f; t.ql[1] = (float)(1.0 - tb); t.ql[2] = (float)tb; t.ql[3] = 0.0f;
    } else {
      t.qh[0] = (float)(1.0 - tb); t.qh[1] = (float)tb; t.qh[2] = 0.0f; t.qh[3] = 0.0f;
      t.ql[0] = t.qh[0]; t.ql[1] = t.qh[1]; t.ql[2] = 0.0f; t.ql[3] = 0.0f;
    }
  }
  t.uniform = uniform_log_knots(pdf->h_x + t.ix0, t.nxs, t.a0, t.inv_da) ? 1 : 0;
  return VGX_OK;
}

// Index of the subgrid holding q2 in a list of subgrids (upper one at a
// threshold, the last closed at its top), -1 if outside.
int subgrid_of(const double* knots, const int* off, const int* nq, int n_sub, double q2) {
  int sub = -1;
  for (int k = 0; k < n_sub; ++k) {
    const double lo = knots[off[k]], hi = knots[off[k] + nq[k] - 1];
    const bool last = k == n_sub - 1;
    if (q2 >= lo && (q2 < hi || (last && q2 <= hi))) sub = k;
  }
  return sub;
}

// cell j with q[j] <= v < q[j+1], clamped to [0, n - 2]
int host_cell(const double* q, int n, double v) {
  int j = 0;
  while (j < n - 2 && q[j + 1] <= v) ++j;
  return j;
}

// t tbar with mu^2 = s_hat/4 per event: the Q^2 rows the scales reach,
// [m_t^2, s/4] plus the stencil margins, and the alpha_s subgrid holding them.
vgx_status setup_ttbar_dynamic(TTDynConst& t, const vgx_pdf* pdf, double rs, double mt, double conv) {
  VGX_CHECK(pdf->n_flav == TT_NF, "TTBAR needs an 11-flavour PDF (order -5..-1, g, 1..5)");
  VGX_CHECK(pdf->n_x <= TT_MAX_NX && pdf->n_x >= 4, "TTBAR supports 4 .. %d x knots", TT_MAX_NX);
  VGX_CHECK(pdf->a_nsub > 0, "TTBAR mode 2 needs an alpha_s table on the PDF (pdf_set_alphas)");
  const double s = rs * rs, tau0 = 4.0 * mt * mt / s;
  VGX_CHECK(tau0 >= pdf->h_x[0], "TTBAR: tau0 below the PDF x range");
  const double mu2_lo = mt * mt, mu2_hi = s / 4.0;
  const int sub = subgrid_of(pdf->h_q2, pdf->q_off, pdf->nq, pdf->n_sub, mu2_lo);
  VGX_CHECK(sub >= 0 && sub == subgrid_of(pdf->h_q2, pdf->q_off, pdf->nq, pdf->n_sub, mu2_hi),
            "TTBAR mode 2: the scales [m_t^2, s/4] must lie in one PDF subgrid");
  const int nq = pdf->nq[sub];
  VGX_CHECK(nq >= 4, "TTBAR mode 2: the PDF subgrid needs at least 4 Q^2 knots");
  const double* q = pdf->h_q2 + pdf->q_off[sub];
  const int jlo = host_cell(q, nq, mu2_lo), jhi = host_cell(q, nq, mu2_hi);
  int r0 = jlo - 1 < nq - 4 ? jlo - 1 : nq - 4;
  r0 = r0 < 0 ? 0 : r0;
  int r1 = jhi + 2 > r0 + 3 ? jhi + 2 : r0 + 3;
  r1 = r1 > nq - 1 ? nq - 1 : r1;
  VGX_CHECK(r1 - r0 + 1 <= TD_MAX_ROWS, "TTBAR mode 2: the scales span more than %d Q^2 rows", TD_MAX_ROWS);
  const int asub = subgrid_of(pdf->h_aq2, pdf->a_off, pdf->a_nq, pdf->a_nsub, mu2_lo);
  VGX_CHECK(asub >= 0 && asub == subgrid_of(pdf->h_aq2, pdf->a_off, pdf->a_nq, pdf->a_nsub, mu2_hi),
            "TTBAR mode 2: the scales [m_t^2, s/4] must lie in one alpha_s subgrid");
  VGX_CHECK(pdf->a_nq[asub] <= TD_MAX_ALPHAS, "TTBAR mode 2: alpha_s subgrid has more than %d knots", TD_MAX_ALPHAS);
  t.L0 = log(1.0 / tau0);
  t.lns4 = log(s / 4.0);
  t.pref = (float)(2.0 * conv / (32.0 * M_PI * s));
  t.v32 = pdf->v32;
  t.fstride = pdf->fstride;
  t.lx = pdf->lx;
  t.n_x = pdf->n_x;
  int i0 = 0;
  while (i0 < pdf->n_x - 2 && pdf->h_x[i0 + 1] <= tau0) ++i0;
  t.ix0 = i0 >= 2 ? i0 - 2 : 0;
  if (pdf->n_x - t.ix0 < 4) t.ix0 = pdf->n_x - 4;
  t.nxs = pdf->n_x - t.ix0;
  t.lq2 = pdf->lq2 + pdf->q_off[sub];
  t.q_glob = pdf->q_off[sub];
  t.nq = nq;
  t.r0 = r0;
  t.R = r1 - r0 + 1;
  t.a_lq2 = pdf->a_lq2 + pdf->a_off[asub];
  t.a_val = pdf->a_val + pdf->a_off[asub];
  t.a_nq = pdf->a_nq[asub];
  t.x_uniform = uniform_log_knots(pdf->h_x + t.ix0, t.nxs, t.a0, t.inv_da) ? 1 : 0;
  t.q_uniform = uniform_log_knots(q + r0, t.R, t.b0, t.inv_db) ? 1 : 0;
  return VGX_OK;
}

// Build the device-side integrand parameters from the user's parameters.
vgx_status prepare_params(vgx_vegas* v, const vgx_vegas_cfg* c) {
  const int d = c->dim;
  double* p = v->prm.p;
  switch (c->kind) {
    case VGX_GAUSS: {
      VGX_CHECK(c->n_params >= 2 * d, "GAUSS needs 2*dim params");
      double norm = 1.0;
      for (int j = 0; j < d; ++j) {
        const double s = c->params[d + j];
        VGX_CHECK(s > 0.0, "GAUSS sigma must be > 0");
        p[j] = c->params[j];
        p[d + j] = 1.0 / (s * sqrt(2.0));
        norm *= 1.0 / (s * sqrt(2.0 * M_PI));
      }
      p[2 * d] = norm;
      return VGX_OK;
    }
    case VGX_GENZ_OSC:
      VGX_CHECK(c->n_params >= 1 + d, "GENZ_OSC needs 1+dim params");
      p[0] = 2.0 * M_PI * c->params[0];
      for (int j = 0; j < d; ++j) p[1 + j] = c->params[1 + j];
      return VGX_OK;
    case VGX_GENZ_PEAK:
      VGX_CHECK(c->n_params >= 2 * d, "GENZ_PEAK needs 2*dim params");
      for (int j = 0; j < d; ++j) {
        const double cj = c->params[d + j];
        VGX_CHECK(cj != 0.0, "GENZ_PEAK c must be non-zero");
        p[j] = c->params[j];
        p[d + j] = 1.0 / (cj * cj);
      }
      return VGX_OK;
    case VGX_TTBAR: {
      VGX_CHECK(d == 3, "TTBAR needs dim 3");
      VGX_CHECK(c->n_params >= 4, "TTBAR needs [sqrt_s, m_top, alpha_s, gev2_to_pb]");
      VGX_CHECK(c->pdf, "TTBAR needs a PDF context");
      const double rs = c->params[0], mt = c->params[1], as = c->params[2], conv = c->params[3];
      VGX_CHECK(rs > 2.0 * mt && mt > 0.0 && as > 0.0, "TTBAR: need sqrt_s > 2 m_top > 0");
      const double s = rs * rs;
      const double tau0 = 4.0 * mt * mt / s;
      const double mode = c->n_params >= 5 ? c->params[4] : 0.0;
      VGX_CHECK(mode == 0.0 || mode == 1.0 || mode == 2.0,
                "TTBAR mode must be 0 (full stencil), 1 (fixed-scale contraction) or 2 (scale per event)");
      if (mode == 2.0) {
        v->tt_dyn = 1;
        return setup_ttbar_dynamic(v->ttd, c->pdf, rs, mt, conv);
      }
      TTbarConst& t = v->tt;
      VGX_TRY(setup_pdf_rows(t.pdf, c->pdf, mt * mt, tau0, mode == 1.0, "TTBAR"));
      t.L0 = log(1.0 / tau0);
      t.pref = (float)(2.0 * conv / (32.0 * M_PI * s));
      t.g4 = (float)((4.0 * M_PI * as) * (4.0 * M_PI * as));
      return VGX_OK;
    }
    case VGX_DRELLYAN: {
      VGX_CHECK(d == 3, "DRELLYAN needs dim 3");
      VGX_CHECK(c->n_params >= 8,
                "DRELLYAN needs [sqrt_s, m_lo, m_hi, m_z, gamma_z, sin2w, alpha, gev2_to_pb]");
      VGX_CHECK(c->pdf, "DRELLYAN needs a PDF context");
      const double* q = c->params;
      const double rs = q[0], mlo = q[1], mhi = q[2], mz = q[3], gz = q[4], sw2 = q[5], al = q[6], conv = q[7];
      VGX_CHECK(mlo > 0.0 && mhi > mlo && mhi < rs, "DRELLYAN: need 0 < m_lo < m_hi < sqrt_s");
      VGX_CHECK(mz > 0.0 && gz > 0.0 && sw2 > 0.0 && sw2 < 1.0 && al > 0.0, "DRELLYAN: bad electroweak inputs");
      const double mode = c->n_params >= 9 ? q[8] : 0.0;
      VGX_CHECK(mode == 0.0 || mode == 1.0, "DRELLYAN mode must be 0 (full stencil) or 1 (fixed-scale contraction)");
      const double s = rs * rs, tlo = mlo * mlo / s, thi = mhi * mhi / s;
      DYConst& t = v->dy;
      VGX_TRY(setup_pdf_rows(t.pdf, c->pdf, mz * mz, tlo, mode == 1.0, "DRELLYAN"));
      t.Llo = log(1.0 / tlo);
      t.Lr = log(thi / tlo);
      t.mlo2 = mlo * mlo;
      t.mz2d = mz * mz;
      // F = J/tau conv dsigma/dcos summed: J/tau = 2 Lr ln(1/tau), dsigma/dcos
      // = (e^4/12) A / (32 pi s_hat)
      const double e4 = (4.0 * M_PI * al) * (4.0 * M_PI * al);
      t.pref = (float)(2.0 * t.Lr * conv * e4 / (12.0 * 32.0 * M_PI));
      t.mg2 = (float)(mz * mz * gz * gz);
      t.kap = (float)(1.0 / (sw2 * (1.0 - sw2)));
      // helicity sums: same (LL + RR) and opposite (LR + RL) helicity pairs,
      // S = a0 + a1 Re chi + a2 |chi|^2, for up- and down-type quarks
      const double ql = -1.0, gll = -0.5 + sw2, grl = sw2;
      for (int k = 0; k < 2; ++k) {
        const double qq = k == 0 ? 2.0 / 3.0 : -1.0 / 3.0, t3 = k == 0 ? 0.5 : -0.5;
        const double glq = t3 - qq * sw2, grq = -qq * sw2;
        const double qq2 = qq * ql;
        t.a0[k] = (float)(2.0 * qq2 * qq2);
        t.as1[k] = (float)(2.0 * qq2 * (glq * gll + grq * grl));
        t.as2[k] = (float)(glq * gll * glq * gll + grq * grl * grq * grl);
        t.ao1[k] = (float)(2.0 * qq2 * (glq * grl + grq * gll));
        t.ao2[k] = (float)(glq * grl * glq * grl + grq * gll * grq * gll);
      }
      return VGX_OK;
    }
    case VGX_SINGLETOP: {
      VGX_CHECK(d == 3, "SINGLETOP needs dim 3");
      VGX_CHECK(c->n_params >= 7, "SINGLETOP needs [sqrt_s, m_top, m_w, gamma_w, sin2w, alpha, gev2_to_pb]");
      VGX_CHECK(c->pdf, "SINGLETOP needs a PDF context");
      const double* q = c->params;
      const double rs = q[0], mt = q[1], mw = q[2], gw = q[3], sw2 = q[4], al = q[5], conv = q[6];
      VGX_CHECK(mt > 0.0 && rs > mt, "SINGLETOP: need sqrt_s > m_top > 0");
      VGX_CHECK(mw > 0.0 && gw > 0.0 && sw2 > 0.0 && sw2 < 1.0 && al > 0.0, "SINGLETOP: bad electroweak inputs");
      const double mode = c->n_params >= 8 ? q[7] : 0.0;
      VGX_CHECK(mode == 0.0 || mode == 1.0, "SINGLETOP mode must be 0 (full stencil) or 1 (fixed-scale contraction)");
      const double s = rs * rs, tau0 = mt * mt / s;
      STConst& t = v->st;
      VGX_TRY(setup_pdf_rows(t.pdf, c->pdf, mt * mt, tau0, mode == 1.0, "SINGLETOP"));
      t.L0 = log(1.0 / tau0);
      t.mt2 = (float)(mt * mt);
      t.mw2 = (float)(mw * mw);
      t.mwg2 = (float)(mw * mw * gw * gw);
      const double g2 = 4.0 * M_PI * al / sw2;
      t.pref = (float)(2.0 * t.L0 * conv * g2 * g2 / (128.0 * M_PI));
      return VGX_OK;
    }
    default:
      set_error("unknown integrand kind %d", c->kind);
      return VGX_EINVAL;
  }
}

double pow_int(double b, int e) {
  double r = 1.0;
  for (int k = 0; k < e; ++k) r *= b;
  return r;
}

// Launch helpers dispatching on (kind, prec, D).
template <int D, class F, class Src, bool HIST>
vgx_status launch_iter_f(vgx_vegas* v, int64_t n, const F& f, const Src& src) {
  VegasArgs a{n, v->edges, v->nb, v->pstride, hist_copies(D, v->nb, !F::kStage), pow_int((double)v->nb, D),
              v->nb * 0x1p-32, v->tables, v->table_bytes};
  const int grid = grid_for(v, n);
  const size_t lds = sizeof(double) * (size_t)lds_table_offset(D, v->nb, HIST, !F::kStage) + extra_lds_bytes(v);
  if (src.seg_len(0, n) == n)  // one segment: the common case
    hipLaunchKernelGGL((k_vegas_iter<D, F, Src, HIST, false>), dim3(grid), dim3(BLOCK), lds, v->stream, a, f, src,
                       v->partials);
  else
    hipLaunchKernelGGL((k_vegas_iter<D, F, Src, HIST, true>), dim3(grid), dim3(BLOCK), lds, v->stream, a, f, src,
                       v->partials);
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

template <int D, class Src, bool HIST>
vgx_status launch_iter_d(vgx_vegas* v, int64_t n, const Src& src) {
  if (v->kind == VGX_TTBAR) {
    if constexpr (D == 3) {
      if (v->tt_dyn) {
        TTbarDyn f{};
        f.c = v->ttd;
        return launch_iter_f<3, TTbarDyn, Src, HIST>(v, n, f, src);
      }
      TTbar f{};
      f.c = v->tt;
      return launch_iter_f<3, TTbar, Src, HIST>(v, n, f, src);
    }
    set_error("TTBAR needs dim 3");
    return VGX_EINVAL;
  }
  if (v->kind == VGX_DRELLYAN) {
    if constexpr (D == 3) {
      DrellYan f{};
      f.c = v->dy;
      return launch_iter_f<3, DrellYan, Src, HIST>(v, n, f, src);
    }
    set_error("DRELLYAN needs dim 3");
    return VGX_EINVAL;
  }
  if (v->kind == VGX_SINGLETOP) {
    if constexpr (D == 3) {
      SingleTop f{};
      f.c = v->st;
      return launch_iter_f<3, SingleTop, Src, HIST>(v, n, f, src);
    }
    set_error("SINGLETOP needs dim 3");
    return VGX_EINVAL;
  }
#define VGX_LAUNCH_KIND(T)                                                     \
  do {                                                                         \
    if (v->prec == VGX_F64) {                                                  \
      T<D, double> f{};                                                        \
      f.prm = v->prm;                                                          \
      return launch_iter_f<D, T<D, double>, Src, HIST>(v, n, f, src);          \
    } else {                                                                   \
      T<D, float> f{};                                                         \
      f.prm = v->prm;                                                          \
      return launch_iter_f<D, T<D, float>, Src, HIST>(v, n, f, src);           \
    }                                                                          \
  } while (0)
  switch (v->kind) {
    case VGX_GAUSS: VGX_LAUNCH_KIND(Gauss);
    case VGX_GENZ_OSC: VGX_LAUNCH_KIND(GenzOsc);
    case VGX_GENZ_PEAK: VGX_LAUNCH_KIND(GenzPeak);
  }
#undef VGX_LAUNCH_KIND
  set_error("unknown kind");
  return VGX_EINVAL;
}

template <int D, class F>
vgx_status launch_sample_f(vgx_vegas* v, int64_t first, int64_t n, int32_t it, const F& f, double* u, double* g) {
  VegasArgs a{n, v->edges, v->nb, v->pstride, hist_copies(D, v->nb, !F::kStage), pow_int((double)v->nb, D),
              v->nb * 0x1p-32, v->tables, v->table_bytes};
  PhiloxSrc<D> src{(uint32_t)it, v->stream_id, (uint32_t)v->seed, (uint32_t)(v->seed >> 32), first};
  const int grid = grid_for(v, n);
  const size_t lds = sizeof(double) * (size_t)lds_table_offset(D, v->nb, false, !F::kStage) + extra_lds_bytes(v);
  hipLaunchKernelGGL((k_vegas_sample<D, F>), dim3(grid), dim3(BLOCK), lds, v->stream, a, f, src, u, g);
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

template <int D>
vgx_status launch_sample_d(vgx_vegas* v, int64_t first, int64_t n, int32_t it, double* u, double* g) {
  if (v->kind == VGX_TTBAR) {
    if constexpr (D == 3) {
      if (v->tt_dyn) {
        TTbarDyn f{};
        f.c = v->ttd;
        return launch_sample_f<3, TTbarDyn>(v, first, n, it, f, u, g);
      }
      TTbar f{};
      f.c = v->tt;
      return launch_sample_f<3, TTbar>(v, first, n, it, f, u, g);
    }
    set_error("TTBAR needs dim 3");
    return VGX_EINVAL;
  }
  if (v->kind == VGX_DRELLYAN) {
    if constexpr (D == 3) {
      DrellYan f{};
      f.c = v->dy;
      return launch_sample_f<3, DrellYan>(v, first, n, it, f, u, g);
    }
    set_error("DRELLYAN needs dim 3");
    return VGX_EINVAL;
  }
  if (v->kind == VGX_SINGLETOP) {
    if constexpr (D == 3) {
      SingleTop f{};
      f.c = v->st;
      return launch_sample_f<3, SingleTop>(v, first, n, it, f, u, g);
    }
    set_error("SINGLETOP needs dim 3");
    return VGX_EINVAL;
  }
#define VGX_SAMPLE_KIND(T)                                                     \
  do {                                                                         \
    if (v->prec == VGX_F64) {                                                  \
      T<D, double> f{};                                                        \
      f.prm = v->prm;                                                          \
      return launch_sample_f<D, T<D, double>>(v, first, n, it, f, u, g);       \
    } else {                                                                   \
      T<D, float> f{};                                                         \
      f.prm = v->prm;                                                          \
      return launch_sample_f<D, T<D, float>>(v, first, n, it, f, u, g);        \
    }                                                                          \
  } while (0)
  switch (v->kind) {
    case VGX_GAUSS: VGX_SAMPLE_KIND(Gauss);
    case VGX_GENZ_OSC: VGX_SAMPLE_KIND(GenzOsc);
    case VGX_GENZ_PEAK: VGX_SAMPLE_KIND(GenzPeak);
  }
#undef VGX_SAMPLE_KIND
  set_error("unknown kind");
  return VGX_EINVAL;
}

#define VGX_DIM_SWITCH(d, CALL)                                                 \
  switch (d) {                                                                 \
    case 1: return CALL(1); case 2: return CALL(2); case 3: return CALL(3);    \
    case 4: return CALL(4); case 5: return CALL(5); case 6: return CALL(6);    \
    case 7: return CALL(7); case 8: return CALL(8); case 9: return CALL(9);    \
    case 10: return CALL(10); case 11: return CALL(11); case 12: return CALL(12); \
  }

vgx_status timed_flush(vgx_vegas* v) {
  for (int k = 0; k < v->t_pending; ++k) {
    VGX_HIP(hipEventSynchronize(v->ev[2 * k + 1]));
    float ms = 0.f;
    VGX_HIP(hipEventElapsedTime(&ms, v->ev[2 * k], v->ev[2 * k + 1]));
    v->t_ms += ms;
    v->t_launches += 1;
  }
  v->t_pending = 0;
  return VGX_OK;
}

// Whether the launch about to be enqueued is one of the timed ones.
bool timed_now(const vgx_vegas* v) { return v->timing && v->t_seen % v->t_every == 0; }

vgx_status timed_begin(vgx_vegas* v) {
  if (!timed_now(v)) return VGX_OK;
  if (v->t_pending == vgx_vegas::kTimerPairs) VGX_TRY(timed_flush(v));
  VGX_HIP(hipEventRecord(v->ev[2 * v->t_pending], v->stream));
  return VGX_OK;
}

vgx_status timed_end(vgx_vegas* v) {
  if (!v->timing) return VGX_OK;
  if (timed_now(v)) {
    VGX_HIP(hipEventRecord(v->ev[2 * v->t_pending + 1], v->stream));
    v->t_pending += 1;
  }
  v->t_seen += 1;
  return VGX_OK;
}

vgx_status launch_philox_iter(vgx_vegas* v, int64_t n, int32_t it) {
#define CALL(D) launch_iter_d<D, PhiloxSrc<D>, true>(v, n, PhiloxSrc<D>{(uint32_t)it, v->stream_id, (uint32_t)v->seed, (uint32_t)(v->seed >> 32), 0})
  VGX_DIM_SWITCH(v->dim, CALL)
#undef CALL
  set_error("bad dim");
  return VGX_EINVAL;
}

vgx_status launch_points_iter(vgx_vegas* v, int64_t n, const double* y, const double* logq) {
#define CALL(D) launch_iter_d<D, PointsSrc<D>, false>(v, n, PointsSrc<D>{y, logq, n})
  VGX_DIM_SWITCH(v->dim, CALL)
#undef CALL
  set_error("bad dim");
  return VGX_EINVAL;
}

// The fused flow-sampling iteration (k_flow_iter) for integrand F; sets the
// grid (the partial rows to reduce).
template <int D, class F>
vgx_status launch_flow_iter_f(vgx_vegas* v, const FlowView& fv, int64_t n, FlowIterArgs fa, const F& f, int* grid) {
  VegasArgs a{n, v->edges, v->nb, v->pstride, 1, pow_int((double)v->nb, D), v->nb * 0x1p-32, v->tables,
              v->table_bytes};
  const size_t base = sizeof(double) * (size_t)lds_table_offset(D, v->nb, false, !F::kStage) + extra_lds_bytes(v);
  const size_t off = (base + 15) & ~(size_t)15;
  const size_t lds = off + fwd_z_offset(fv.fw_total, fv.bias_total, 2) + sizeof(float) * (size_t)D * FI_BLOCK;
  VGX_CHECK(lds <= 160 * 1024, "flow_vegas_iterate: the flow's weights and the integrand's tables need %zu bytes of LDS",
            lds);
  fa.flow_off = (int)off;
  const void* k = reinterpret_cast<const void*>(&k_flow_iter<D, F, OpBF16>);
  static size_t allowed = 0;  // per instantiation: the dynamic LDS allowed so far (never lowered)
  if (lds > allowed) {
    VGX_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    allowed = lds;
  }
  // one workgroup per CU (the LDS), at most one tile pair per wave and round
  const int64_t pairs = (n + 63) / 64;
  int64_t g = device_cus();
  if (g > v->max_wg) g = v->max_wg;
  if (g * (FI_BLOCK / 64) > pairs) g = (pairs + FI_BLOCK / 64 - 1) / (FI_BLOCK / 64);
  *grid = (int)(g < 1 ? 1 : g);
  hipLaunchKernelGGL((k_flow_iter<D, F, OpBF16>), dim3(*grid), dim3(FI_BLOCK), lds, v->stream, a, f, fa, v->partials);
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

template <int D>
vgx_status launch_flow_iter_d(vgx_vegas* v, const FlowView& fv, int64_t n, const FlowIterArgs& fa, int* grid) {
  if constexpr (D == 3) {
    if (v->kind == VGX_TTBAR) {
      if (v->tt_dyn) {
        TTbarDyn f{};
        f.c = v->ttd;
        return launch_flow_iter_f<3, TTbarDyn>(v, fv, n, fa, f, grid);
      }
      TTbar f{};
      f.c = v->tt;
      return launch_flow_iter_f<3, TTbar>(v, fv, n, fa, f, grid);
    }
    if (v->kind == VGX_DRELLYAN) {
      DrellYan f{};
      f.c = v->dy;
      return launch_flow_iter_f<3, DrellYan>(v, fv, n, fa, f, grid);
    }
    if (v->kind == VGX_SINGLETOP) {
      SingleTop f{};
      f.c = v->st;
      return launch_flow_iter_f<3, SingleTop>(v, fv, n, fa, f, grid);
    }
  }
#define VGX_FLOW_KIND(T)                                                       \
  do {                                                                         \
    if (v->prec == VGX_F64) {                                                  \
      T<D, double> f{};                                                        \
      f.prm = v->prm;                                                          \
      return launch_flow_iter_f<D, T<D, double>>(v, fv, n, fa, f, grid);       \
    } else {                                                                   \
      T<D, float> f{};                                                         \
      f.prm = v->prm;                                                          \
      return launch_flow_iter_f<D, T<D, float>>(v, fv, n, fa, f, grid);        \
    }                                                                          \
  } while (0)
  switch (v->kind) {
    case VGX_GAUSS: VGX_FLOW_KIND(Gauss);
    case VGX_GENZ_OSC: VGX_FLOW_KIND(GenzOsc);
    case VGX_GENZ_PEAK: VGX_FLOW_KIND(GenzPeak);
  }
#undef VGX_FLOW_KIND
  set_error("flow_vegas_iterate: integrand kind %d needs a different dimension", v->kind);
  return VGX_EINVAL;
}

vgx_status launch_flow_iter(vgx_vegas* v, const FlowView& fv, int64_t n, const FlowIterArgs& fa, int* grid) {
  switch (v->dim) {
    case 2: return launch_flow_iter_d<2>(v, fv, n, fa, grid);
    case 3: return launch_flow_iter_d<3>(v, fv, n, fa, grid);
    case 4: return launch_flow_iter_d<4>(v, fv, n, fa, grid);
    case 5: return launch_flow_iter_d<5>(v, fv, n, fa, grid);
    case 6: return launch_flow_iter_d<6>(v, fv, n, fa, grid);
    case 7: return launch_flow_iter_d<7>(v, fv, n, fa, grid);
    case 8: return launch_flow_iter_d<8>(v, fv, n, fa, grid);
  }
  set_error("flow_vegas_iterate: dimension %d (the fused iteration takes 2..8)", v->dim);
  return VGX_EINVAL;
}

vgx_status launch_sample(vgx_vegas* v, int64_t first, int64_t n, int32_t it, double* u, double* g) {
#define CALL(D) launch_sample_d<D>(v, first, n, it, u, g)
  VGX_DIM_SWITCH(v->dim, CALL)
#undef CALL
  set_error("bad dim");
  return VGX_EINVAL;
}

// Reduce the partial rows into the histogram and record n_rec.  With defer,
// the record keeps only S1 and S2 until vegas_refine or vegas_flush_pending
// completes it (the context notes it as pending).
vgx_status launch_reduce(vgx_vegas* v, int rows, int ncols, int64_t n, bool defer = false) {
  VGX_CHECK(rows >= 1 && rows <= RMAXROWS, "reduce: %d partial rows (1..%d)", rows, RMAXROWS);
  VGX_CHECK(v->pend_k < 0, "reduce: record %d is still pending", v->pend_k);
  const int blocks = (ncols + RCOLS - 1) / RCOLS;
  hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(RBLOCK), 0, v->stream, v->partials, rows, v->pstride, ncols,
                     v->hist, n, v->rec, v->n_rec, v->comb, defer ? 1 : 0);
  VGX_HIP(hipGetLastError());
  if (defer) {
    v->pend_k = v->n_rec;
    v->pend_n = n;
  }
  return VGX_OK;
}

// What produced a record: the context's own sampling (plain VEGAS), caller
// points with q = 1, or caller points from a proposal with density q.
enum RecordKind { REC_PLAIN = 0, REC_POINTS = 1, REC_PROPOSAL = 2 };

// Record k and the combination in one round trip: a later vegas_result
// reads the combination from the host copy until new records are enqueued.
// Plain VEGAS judges a proposal: a finite proposal estimate whose variance
// per sample, n var(E), exceeds that of the latest plain iteration read
// back returns VGX_EFALLBACK (the estimate is unbiased and stays recorded).
// With VGX_TRACE set to a file name ("-": standard error), every estimate
// read back is appended there as one JSON line: the record, the combination
// after it, and an FNV-1a hash of the grid it was sampled on.
void trace_record(vgx_vegas* v, int k, const IterRecord* h, const Combined* hc, RecordKind kind) {
  const char* path = getenv("VGX_TRACE");
  if (!path || !*path) return;
  const size_t ne = (size_t)v->dim * (v->nb + 1);
  double* g = (double*)((char*)v->pinned + sizeof(IterRecord) * MAX_RECORDS + sizeof(Combined));
  uint64_t hash = 14695981039346656037ull;
  if (hipMemcpyAsync(g, v->edges, sizeof(double) * ne, hipMemcpyDeviceToHost, v->stream) == hipSuccess &&
      hipStreamSynchronize(v->stream) == hipSuccess) {
    const unsigned char* b = (const unsigned char*)g;
    for (size_t i = 0; i < sizeof(double) * ne; ++i) hash = (hash ^ b[i]) * 1099511628211ull;
  } else {
    (void)hipGetLastError();
    hash = 0;
  }
  static const char* kinds[] = {"plain", "points", "proposal"};
  const bool err = strcmp(path, "-") == 0;
  FILE* fp = err ? stderr : fopen(path, "a");
  if (!fp) return;
  fprintf(fp,
          "{\"context\": \"%p\", \"record\": %d, \"kind\": \"%s\", \"n\": %lld, \"mean\": %.17g, \"var\": %.17g, "
          "\"finite\": %d, \"combined_mean\": %.17g, \"combined_sigma\": %.17g, \"chi2_dof\": %.17g, "
          "\"records_used\": %d, \"grid_fnv1a\": \"%016llx\"}\n",
          (void*)v, k, kinds[kind], (long long)h->n, h->mean, h->var, (int)h->finite, hc->mean, hc->sigma, hc->chi2_dof,
          (int)hc->n_used, (unsigned long long)hash);
  if (err) fflush(fp);
  else fclose(fp);
}

vgx_status read_record(vgx_vegas* v, int k, vgx_iter_result* out, RecordKind kind) {
  IterRecord* h = (IterRecord*)v->pinned;
  Combined* hc = (Combined*)((char*)v->pinned + sizeof(IterRecord) * MAX_RECORDS);
  VGX_HIP(hipMemcpyAsync(h, v->rec + k, sizeof(IterRecord), hipMemcpyDeviceToHost, v->stream));
  VGX_HIP(hipMemcpyAsync(hc, v->comb, sizeof(Combined), hipMemcpyDeviceToHost, v->stream));
  VGX_HIP(hipStreamSynchronize(v->stream));
  v->comb_fresh = true;
  trace_record(v, k, h, hc, kind);
  if (out) {
    out->mean = h->mean;
    out->var = h->var;
    out->s1 = h->s1;
    out->s2 = h->s2;
    out->n = h->n;
  }
  if (!h->finite) {
    set_error("non-finite iteration estimate (mean=%g var=%g); excluded from the combination", h->mean, h->var);
    return VGX_ENUMERIC;
  }
  const double per_sample = h->var * (double)h->n;
  if (kind == REC_PLAIN) v->judge_var = per_sample;
  if (kind == REC_PROPOSAL && v->judge_var >= 0.0 && per_sample > v->judge_var) {
    set_error("proposal variance per sample %.6g exceeds plain VEGAS's %.6g: fall back to VEGAS", per_sample,
              v->judge_var);
    return VGX_EFALLBACK;
  }
  return VGX_OK;
}

}  // namespace

vgx_status vegas_flush_pending(vgx_vegas* v) {
  if (v->pend_k < 0) return VGX_OK;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, v->stream, v->rec, v->pend_k, v->pend_n, v->comb);
  VGX_HIP(hipGetLastError());
  v->pend_k = -1;
  return VGX_OK;
}

extern "C" vgx_status vegas_create(const vgx_vegas_cfg* c, void* stream, vgx_vegas** out) {
  VGX_CHECK(c && out, "vegas_create: null argument");
  *out = nullptr;
  VGX_CHECK(c->dim >= 1 && c->dim <= VGX_MAX_DIM, "vegas_create: dim %d out of 1..%d", c->dim, VGX_MAX_DIM);
  VGX_CHECK(c->n_bins >= 2 && c->n_bins <= VGX_MAX_BINS, "vegas_create: n_bins %d out of 2..%d", c->n_bins,
            VGX_MAX_BINS);
  VGX_CHECK(c->prec == VGX_F64 || c->prec == VGX_F32, "vegas_create: bad prec");
  VGX_CHECK(c->alpha >= 0.0 && c->alpha < 100.0, "vegas_create: bad alpha");
  VGX_CHECK(c->stream_id < (1u << 23), "vegas_create: stream_id must be < 2^23");
  VGX_CHECK(c->n_params <= MAX_PARAMS && (c->n_params == 0 || c->params), "vegas_create: bad params");
  vgx_vegas* v = new vgx_vegas();
  hipGetDevice(&v->device);
  v->stream = (hipStream_t)stream;
  v->kind = c->kind;
  v->dim = c->dim;
  v->nb = c->n_bins;
  v->prec = c->prec;
  v->alpha = c->alpha;
  v->seed = c->seed;
  v->stream_id = c->stream_id;
  vgx_status s = prepare_params(v, c);
  if (s != VGX_OK) { delete v; return s; }
  v->max_wg = device_cus() * (uses_pdf(c->kind) ? hadronic_blocks_per_cu(v) : 8);
  v->max_wg = v->max_wg < RMAXROWS ? v->max_wg : RMAXROWS;  // rows one reduction takes
  v->pstride = 4 + v->dim * v->nb;
  const size_t ne = (size_t)v->dim * (v->nb + 1);
  do {
    if ((s = dev_alloc((void**)&v->edges, sizeof(double) * ne)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&v->hist, sizeof(double) * v->dim * v->nb)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&v->partials, sizeof(double) * (size_t)v->max_wg * v->pstride)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&v->rec, sizeof(IterRecord) * MAX_RECORDS)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&v->comb, sizeof(Combined))) != VGX_OK) break;
    if ((s = host_alloc(&v->pinned, sizeof(IterRecord) * MAX_RECORDS + sizeof(Combined) + sizeof(double) * ne)) != VGX_OK) break;
    if ((s = build_tables(v)) != VGX_OK) break;
  } while (0);
  if (s != VGX_OK) { vegas_destroy(v); return s; }
  double* h = (double*)v->pinned;
  for (int j = 0; j < v->dim; ++j)
    for (int k = 0; k <= v->nb; ++k) h[j * (v->nb + 1) + k] = (double)k / (double)v->nb;
  hipError_t e = hipMemcpyAsync(v->edges, h, sizeof(double) * ne, hipMemcpyHostToDevice, v->stream);
  if (e == hipSuccess) e = hipMemsetAsync(v->hist, 0, sizeof(double) * v->dim * v->nb, v->stream);
  if (e == hipSuccess) e = hipMemsetAsync(v->comb, 0, sizeof(Combined), v->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(v->stream);
  if (e != hipSuccess) { s = hip_fail(e, "vegas_create init", __FILE__, __LINE__); vegas_destroy(v); return s; }
  *out = v;
  return VGX_OK;
}

static vgx_status iterate_enqueue(vgx_vegas* v, int64_t n, int32_t iteration, bool defer) {
  VGX_CHECK(v, "vegas_iterate: null context");
  VGX_CHECK(n >= 2, "vegas_iterate: need n >= 2 samples");
  if (v->n_rec >= MAX_RECORDS) { set_error("vegas_iterate: more than %d stored estimates", MAX_RECORDS); return VGX_ESTATE; }
  VGX_TRY(vegas_flush_pending(v));
  VGX_TRY(timed_begin(v));
  VGX_TRY(launch_philox_iter(v, n, iteration));
  VGX_TRY(timed_end(v));
  VGX_TRY(launch_reduce(v, grid_for(v, n), v->pstride, n, defer));
  v->have_hist = true;
  return VGX_OK;
}

extern "C" vgx_status vegas_iterate(vgx_vegas* v, int64_t n, int32_t iteration, vgx_iter_result* out) {
  VGX_TRY(iterate_enqueue(v, n, iteration, false));
  v->comb_fresh = false;
  const int k = v->n_rec++;
  return read_record(v, k, out, REC_PLAIN);
}

extern "C" vgx_status vegas_iterate_async(vgx_vegas* v, int64_t n, int32_t iteration) {
  VGX_TRY(iterate_enqueue(v, n, iteration, true));
  v->comb_fresh = false;
  v->n_rec++;
  return VGX_OK;
}

extern "C" vgx_status vegas_refine(vgx_vegas* v) {
  VGX_CHECK(v, "vegas_refine: null context");
  if (!v->have_hist) { set_error("vegas_refine: no histogram (run vegas_iterate first)"); return VGX_ESTATE; }
  const int kp = v->pend_k;
  hipLaunchKernelGGL(k_refine, dim3(v->dim + (kp >= 0 ? 1 : 0)), dim3(64), 0, v->stream, v->edges, v->hist, v->nb,
                     v->alpha, v->rec, kp, v->pend_n, v->comb);
  VGX_HIP(hipGetLastError());
  v->pend_k = -1;
  return VGX_OK;
}

extern "C" vgx_status vegas_result(vgx_vegas* v, double* mean, double* sigma, double* chi2, int32_t* n_used) {
  VGX_CHECK(v, "vegas_result: null context");
  Combined* h = (Combined*)((char*)v->pinned + sizeof(IterRecord) * MAX_RECORDS);
  if (v->n_rec == 0) {
    if (mean) *mean = 0.0;
    if (sigma) *sigma = 0.0;
    if (chi2) *chi2 = 0.0;
    if (n_used) *n_used = 0;
    return VGX_OK;
  }
  VGX_TRY(vegas_flush_pending(v));
  if (!v->comb_fresh) {
    VGX_HIP(hipMemcpyAsync(h, v->comb, sizeof(Combined), hipMemcpyDeviceToHost, v->stream));
    VGX_HIP(hipStreamSynchronize(v->stream));
    v->comb_fresh = true;
  }
  if (mean) *mean = h->mean;
  if (sigma) *sigma = h->sigma;
  if (chi2) *chi2 = h->chi2_dof;
  if (n_used) *n_used = h->n_used;
  return VGX_OK;
}

extern "C" vgx_status vegas_results(vgx_vegas* v, vgx_iter_result* out, int32_t cap, int32_t* count) {
  VGX_CHECK(v && count && (cap == 0 || out), "vegas_results: bad argument");
  const int m = v->n_rec < cap ? v->n_rec : cap;
  IterRecord* h = (IterRecord*)v->pinned;
  VGX_TRY(vegas_flush_pending(v));
  if (m > 0) {
    VGX_HIP(hipMemcpyAsync(h, v->rec, sizeof(IterRecord) * m, hipMemcpyDeviceToHost, v->stream));
    VGX_HIP(hipStreamSynchronize(v->stream));
  }
  for (int k = 0; k < m; ++k) {
    out[k].mean = h[k].mean;
    out[k].var = h[k].var;
    out[k].s1 = h[k].s1;
    out[k].s2 = h[k].s2;
    out[k].n = h[k].n;
  }
  *count = v->n_rec;
  return VGX_OK;
}

extern "C" vgx_status vegas_reset_results(vgx_vegas* v) {
  VGX_CHECK(v, "vegas_reset_results: null context");
  v->pend_k = -1;  // a record still pending is discarded with the rest
  v->n_rec = 0;
  v->comb_fresh = false;
  VGX_HIP(hipMemsetAsync(v->comb, 0, sizeof(Combined), v->stream));
  return VGX_OK;
}

extern "C" vgx_status vegas_get_grid(vgx_vegas* v, double* edges) {
  VGX_CHECK(v && edges, "vegas_get_grid: null argument");
  VGX_HIP(hipMemcpyAsync(edges, v->edges, sizeof(double) * v->dim * (v->nb + 1), hipMemcpyDeviceToHost, v->stream));
  VGX_HIP(hipStreamSynchronize(v->stream));
  return VGX_OK;
}

extern "C" vgx_status vegas_set_grid(vgx_vegas* v, const double* edges) {
  VGX_CHECK(v && edges, "vegas_set_grid: null argument");
  for (int j = 0; j < v->dim; ++j) {
    const double* e = edges + (size_t)j * (v->nb + 1);
    VGX_CHECK(e[0] == 0.0 && e[v->nb] == 1.0, "vegas_set_grid: edges of dim %d must span [0, 1]", j);
    for (int k = 0; k < v->nb; ++k) VGX_CHECK(e[k + 1] > e[k], "vegas_set_grid: edges of dim %d not increasing", j);
  }
  const size_t bytes = sizeof(double) * v->dim * (v->nb + 1);
  double* h = (double*)((char*)v->pinned + sizeof(IterRecord) * MAX_RECORDS + sizeof(Combined));
  VGX_HIP(hipStreamSynchronize(v->stream));
  memcpy(h, edges, bytes);
  VGX_HIP(hipMemcpyAsync(v->edges, h, bytes, hipMemcpyHostToDevice, v->stream));
  VGX_HIP(hipStreamSynchronize(v->stream));
  return VGX_OK;
}

extern "C" vgx_status vegas_get_hist(vgx_vegas* v, double* hist) {
  VGX_CHECK(v && hist, "vegas_get_hist: null argument");
  VGX_HIP(hipMemcpyAsync(hist, v->hist, sizeof(double) * v->dim * v->nb, hipMemcpyDeviceToHost, v->stream));
  VGX_HIP(hipStreamSynchronize(v->stream));
  return VGX_OK;
}

extern "C" vgx_status vegas_sample(vgx_vegas* v, int64_t first, int64_t n, int32_t iteration, double* u, double* g) {
  VGX_CHECK(v, "vegas_sample: null context");
  VGX_CHECK(n >= 0 && first >= 0, "vegas_sample: negative range");
  if (n == 0 || (!u && !g)) return VGX_OK;
  return launch_sample(v, first, n, iteration, u, g);
}

extern "C" vgx_status vegas_iterate_points(vgx_vegas* v, int64_t n, const double* y, const double* logq,
                                           vgx_iter_result* out) {
  VGX_CHECK(v, "vegas_iterate_points: null context");
  VGX_CHECK(n >= 2 && y, "vegas_iterate_points: need n >= 2 and points");
  if (v->n_rec >= MAX_RECORDS) { set_error("vegas_iterate_points: too many stored estimates"); return VGX_ESTATE; }
  VGX_TRY(vegas_flush_pending(v));
  VGX_TRY(timed_begin(v));
  VGX_TRY(launch_points_iter(v, n, y, logq));
  VGX_TRY(timed_end(v));
  VGX_TRY(launch_reduce(v, grid_for(v, n), 4, n));
  v->comb_fresh = false;
  const int k = v->n_rec++;
  return read_record(v, k, out, logq ? REC_PROPOSAL : REC_POINTS);
}

extern "C" vgx_status flow_vegas_iterate(vgx_flow* f, vgx_vegas* v, int64_t n, uint64_t seed, uint32_t stream_id,
                                         int32_t iteration, vgx_iter_result* out) {
  VGX_CHECK(f && v, "flow_vegas_iterate: null flow or context");
  VGX_CHECK(n >= 2, "flow_vegas_iterate: need n >= 2");
  VGX_CHECK(stream_id < (1u << 23), "flow_vegas_iterate: stream_id >= 2^23");
  const FlowView fv = flow_view(f);
  VGX_CHECK(fv.dim == v->dim, "flow_vegas_iterate: flow dimension %d, context dimension %d", fv.dim, v->dim);
  VGX_CHECK(!fv.f32ops, "flow_vegas_iterate: the flow runs FP32 validation operands (the fused iteration takes BF16)");
  if (v->n_rec >= MAX_RECORDS) { set_error("flow_vegas_iterate: too many stored estimates"); return VGX_ESTATE; }
  FlowIterArgs fa{fv.desc, fv.fw, fv.bias, 0, (uint32_t)iteration, stream_id | (1u << 23), (uint32_t)seed,
                  (uint32_t)(seed >> 32)};
  VGX_TRY(vegas_flush_pending(v));
  VGX_TRY(flow_order_before(f, v->stream));
  VGX_TRY(timed_begin(v));
  int grid = 0;
  VGX_TRY(launch_flow_iter(v, fv, n, fa, &grid));
  VGX_TRY(timed_end(v));
  VGX_TRY(launch_reduce(v, grid, 4, n));
  v->comb_fresh = false;
  const int k = v->n_rec++;
  return read_record(v, k, out, REC_PROPOSAL);
}

extern "C" void* vegas_stream(vgx_vegas* v) { return v ? (void*)v->stream : nullptr; }

extern "C" vgx_status vegas_shape(const vgx_vegas* v, int32_t* dim, int32_t* n_bins) {
  VGX_CHECK(v, "vegas_shape: null context");
  if (dim) *dim = v->dim;
  if (n_bins) *n_bins = v->nb;
  return VGX_OK;
}

extern "C" vgx_status vegas_set_timing(vgx_vegas* v, int32_t every) {
  VGX_CHECK(v, "vegas_set_timing: null context");
  VGX_CHECK(every >= 0, "vegas_set_timing: every must be >= 0");
  const int enable = every > 0;
  if (enable && !v->ev[0]) {
    // the events only time: no system-scope fence (cache write-back and
    // invalidation) at each record, which would slow the work they bracket
    for (int k = 0; k < 2 * vgx_vegas::kTimerPairs; ++k)
      VGX_HIP(hipEventCreateWithFlags(&v->ev[k], hipEventDisableSystemFence));
  }
  v->timing = enable != 0;
  v->t_every = enable ? every : 1;
  v->t_seen = 0;
  v->t_pending = 0;
  v->t_ms = 0.0;
  v->t_launches = 0;
  return VGX_OK;
}

extern "C" vgx_status vegas_kernel_time(vgx_vegas* v, double* ms, int64_t* launches) {
  VGX_CHECK(v && ms && launches, "vegas_kernel_time: null argument");
  VGX_TRY(timed_flush(v));
  *ms = v->t_ms;
  *launches = v->t_launches;
  return VGX_OK;
}

extern "C" void vegas_destroy(vgx_vegas* v) {
  if (!v) return;
  if (v->stream) hipStreamSynchronize(v->stream);
  hipFree(v->edges);
  hipFree(v->hist);
  hipFree(v->partials);
  hipFree(v->tables);
  hipFree(v->rec);
  hipFree(v->comb);
  if (v->pinned) hipHostFree(v->pinned);
  for (int k = 0; k < 2 * vgx_vegas::kTimerPairs; ++k)
    if (v->ev[k]) hipEventDestroy(v->ev[k]);
  delete v;
}
