// Log-bicubic PDF interpolation on subgrids (LHAPDF-style), FP64 arithmetic,
// FP64 or FP32 output; every member of a PDF set at once (k_pdf_members).
//
// Thesis: PDF chapter, LHAPDF paragraphs (knots in (x, Q^2), subgrids split
// at quark-mass thresholds, cubic Hermite in (log x, log Q) on 4 neighbouring
// knots, bilinear where the 4-knot stencil is unavailable) and PDFFlow's
// Subgrid design.  The Hermite node slopes are the average of the two
// adjacent secants (LHAPDF6's rule, Buckley et al. 2015).
//
// Kernel design (MI355X): the cubic Hermite with secant slopes is linear in
// the four node values, so for a query the 4x4 stencil reduces to 16
// weights w_rk = q_r c_k computed once and shared by all flavours; node
// values are stored [iq][ix][flav] so that one stencil row (4 consecutive x
// knots) is one contiguous 4*n_flav run.  Knots are staged in LDS for the
// binary searches; outputs are written structure-of-arrays, coalesced.
#include "pdf_internal.h"

#include <float.h>
#include <math.h>
#include <type_traits>
#include <stdlib.h>

namespace vgx {

struct PdfKernelArgs {
  int n_x, n_sub, n_flav;
  int nq[VGX_MAX_SUB];
  int q_off[VGX_MAX_SUB + 1];
  double q2_lo[VGX_MAX_SUB], q2_hi[VGX_MAX_SUB];
};

// Weights (cm, c0, c1, c2) of the nodes k-1, k, k+1, k+2 such that
// sum c * F equals the cubic Hermite between k and k+1 at fraction t with
// node slopes the average of adjacent secants.  rm = h_k/h_{k-1},
// rp = h_k/h_{k+1} with h the knot spacings.
__device__ __forceinline__ void hermite_weights(double t, double rm, double rp, double (&c)[4]) {
  const double t2 = t * t, t3 = t2 * t;
  const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
  const double h10 = t3 - 2.0 * t2 + t;
  const double h01 = -2.0 * t3 + 3.0 * t2;
  const double h11 = t3 - t2;
  // d0 = (F1 - F0)/2 + rm (F0 - Fm)/2,  d1 = rp (F2 - F1)/2 + (F1 - F0)/2
  c[0] = -0.5 * h10 * rm;
  c[1] = h00 - 0.5 * h10 + 0.5 * h10 * rm - 0.5 * h11;
  c[2] = h01 + 0.5 * h10 - 0.5 * h11 * rp + 0.5 * h11;
  c[3] = 0.5 * h11 * rp;
}

// first index i in [lo, hi) with key < a[i+1], i.e. a[i] <= key < a[i+1],
// clamped to hi - 1 (so the top knot maps to the last cell).
__device__ __forceinline__ int find_cell(const double* a, int n, double key) {
  int lo = 0, hi = n - 1;  // answer in [0, n-2]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= key) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Outside the grid (thesis PDF chapter, LHAPDF extrapolation paragraphs).
// FREEZE interpolates at the nearest grid point.  CONTINUE is the legacy
// continuation, one flavour at a time (the path is rare, registers matter):
//   low x:   straight line in ln x through the values at x_0 and x_1 at the
//            query's Q^2 -- through ln xf when both exceed 1e-3, else xf;
//   high Q^2: the same in ln Q^2 through the top subgrid's last two rows;
//   low Q^2: xf = G0 r^((gamma - 1) r + 1), r = Q^2/Q^2_min, with gamma the
//            logarithmic derivative d ln xf/d ln Q^2 at Q^2_min of what the
//            grid gives just above it (lowest bilinear cell, or its low-x
//            continuation), which keeps ln xf C^1 across Q^2_min;
//   both outside: x rule first, on the rows the Q^2 rule reads.
// Rows are read with their edge cells' rule: linear in ln x.
// ---------------------------------------------------------------------------
constexpr double kPositive = 1e-3;

// Fraction t of the line through (0, y0), (1, y1): in ln y when both
// values exceed 1e-3, else in y.
__device__ __forceinline__ double continue_line(double t, double y0, double y1) {
  if (y0 > kPositive && y1 > kPositive) {
    const double l0 = log(y0);
    return exp(l0 + t * (log(y1) - l0));
  }
  return y0 + t * (y1 - y0);
}

template <typename ValT>
__device__ __forceinline__ double node_val(const ValT* vals, int n_x, int nf, int row, int ix, int f) {
  return (double)vals[((int64_t)row * n_x + ix) * nf + f];
}

// Flavour f on global row `row` at ln x = a (cell i, x_0 <= x), linear in a;
// below x_0 (i < 0) the low-x line through the row's first two nodes.
template <typename ValT>
__device__ double row_value(const ValT* vals, const double* slx, int n_x, int nf, int row, int i, double a, int f) {
  if (i < 0)
    return continue_line((a - slx[0]) / (slx[1] - slx[0]), node_val(vals, n_x, nf, row, 0, f),
                         node_val(vals, n_x, nf, row, 1, f));
  const double t = (a - slx[i]) / (slx[i + 1] - slx[i]);
  const double v0 = node_val(vals, n_x, nf, row, i, f), v1 = node_val(vals, n_x, nf, row, i + 1, f);
  return v0 + t * (v1 - v0);
}

// The interpolator's value for flavour f in cell (i, j) of subgrid s at
// (a, b) = (ln x, ln Q^2): the same weights and summation order as
// k_pdf_interp.
template <typename ValT>
__device__ double cell_value(const PdfKernelArgs& g, const ValT* vals, const double* slx, const double* slq2, int nf,
                             int s, int i, int j, double a, double b, int f) {
  const int nq = g.nq[s];
  const double* lq = slq2 + g.q_off[s];
  const ValT* V = vals + (int64_t)g.q_off[s] * g.n_x * nf;
  double acc = 0.0;
  if (i >= 1 && i <= g.n_x - 3 && j >= 1 && j <= nq - 3) {
    const double ha = slx[i + 1] - slx[i];
    const double hb = lq[j + 1] - lq[j];
    double cx[4], cq[4];
    hermite_weights((a - slx[i]) / ha, ha / (slx[i] - slx[i - 1]), ha / (slx[i + 2] - slx[i + 1]), cx);
    hermite_weights((b - lq[j]) / hb, hb / (lq[j] - lq[j - 1]), hb / (lq[j + 2] - lq[j + 1]), cq);
    for (int r = 0; r < 4; ++r)
      for (int k = 0; k < 4; ++k)
        acc = fma(cq[r] * cx[k], (double)V[((int64_t)(j - 1 + r) * g.n_x + (i - 1 + k)) * nf + f], acc);
  } else {
    const double ta = (a - slx[i]) / (slx[i + 1] - slx[i]);
    const double tb = (b - lq[j]) / (lq[j + 1] - lq[j]);
    const double w[4] = {(1.0 - ta) * (1.0 - tb), ta * (1.0 - tb), (1.0 - ta) * tb, ta * tb};
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 2; ++k)
        acc = fma(w[2 * r + k], (double)V[((int64_t)(j + r) * g.n_x + (i + k)) * nf + f], acc);
  }
  return acc;
}

// CONTINUE value of flavour f at a point outside the grid with 0 < x <= x_max
// and Q^2 > 0; s = subgrid holding Q^2 (or -1), i = x cell (-1 below x_0).
template <typename ValT>
__device__ double continue_value(const PdfKernelArgs& g, const ValT* vals, const double* sx, const double* slx,
                                 const double* sq2, const double* slq2, int nf, int s, int i, double x, double q2,
                                 int f) {
  const double a = log(x), b = log(q2);
  if (s >= 0) {  // low x only: the interpolator at (x_0, Q^2) and (x_1, Q^2)
    const int j = find_cell(sq2 + g.q_off[s], g.nq[s], q2);
    const int i1 = g.n_x > 2 ? 1 : 0;
    const double f0 = cell_value(g, vals, slx, slq2, nf, s, 0, j, slx[0], b, f);
    const double f1 = cell_value(g, vals, slx, slq2, nf, s, i1, j, slx[1], b, f);
    return continue_line((a - slx[0]) / (slx[1] - slx[0]), f0, f1);
  }
  if (q2 > g.q2_hi[g.n_sub - 1]) {  // high Q^2: the top subgrid's last two rows
    const int r1 = g.q_off[g.n_sub] - 1, r0 = r1 - 1;
    const double g0 = row_value(vals, slx, g.n_x, nf, r0, i, a, f);
    const double g1 = row_value(vals, slx, g.n_x, nf, r1, i, a, f);
    return continue_line((b - slq2[r0]) / (slq2[r1] - slq2[r0]), g0, g1);
  }
  // low Q^2: the lowest subgrid's first two rows (global rows 0 and 1)
  const double db = slq2[1] - slq2[0];
  double G0, gamma;
  if (i >= 0) {
    G0 = row_value(vals, slx, g.n_x, nf, 0, i, a, f);
    if (G0 == 0.0) return 0.0;
    gamma = (row_value(vals, slx, g.n_x, nf, 1, i, a, f) - G0) / (db * G0);
  } else {
    const double f0 = node_val(vals, g.n_x, nf, 0, 0, f), f1 = node_val(vals, g.n_x, nf, 0, 1, f);
    const double d0 = (node_val(vals, g.n_x, nf, 1, 0, f) - f0) / db;
    const double d1 = (node_val(vals, g.n_x, nf, 1, 1, f) - f1) / db;
    const double t = (a - slx[0]) / (slx[1] - slx[0]);
    G0 = continue_line(t, f0, f1);
    if (G0 == 0.0) return 0.0;
    gamma = (f0 > kPositive && f1 > kPositive) ? (1.0 - t) * d0 / f0 + t * d1 / f1
                                               : ((1.0 - t) * d0 + t * d1) / G0;
  }
  const double r = q2 / sq2[0];
  return G0 * exp(((gamma - 1.0) * r + 1.0) * (b - slq2[0]));
}

// Per-query LDS slot of the interpolation kernel, in doubles: the stencil's
// x weights [0..3], Q^2 weights [4..7] and a tag [8] (node offset and
// stencil kind), overwritten by the nf sums; an odd count spreads the slots
// of consecutive lanes over the LDS banks.
__host__ __device__ constexpr int pdf_slot_doubles(int nf) { return (nf > 9 ? nf : 9) | 1; }

// Dynamic LDS of the interpolation kernel in bytes: the knots (x, ln x, Q^2,
// ln Q^2) and a slot per query of each wave.
constexpr int kInterpBlock = 256;
constexpr size_t kMaxLds = 65536;
inline size_t pdf_interp_lds_bytes(int n_x, int n_q_total, int nf) {
  return sizeof(double) * (2 * (size_t)n_x + 2 * (size_t)n_q_total + (size_t)kInterpBlock * pdf_slot_doubles(nf));
}

// Tag of a query's slot: >= 0: 2 * (offset of the stencil's first node) +
// (1 for the 4x4 Hermite stencil, 0 for the bilinear 2x2); < 0: no sums.
constexpr int64_t kTagNaN = -1;    // outside the grid: NaN outputs
constexpr int64_t kTagSkip = -2;   // outside, written by the continuation pass
constexpr int64_t kTagNone = -3;   // past the last query

// Orders the LDS writes of some lanes of a wave before the reads of others.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The interpolation kernel.  NF > 0: compile-time flavour count; NF == 0:
// run-time count (<= VGX_MAX_FLAV).  ValT: node-value type read from memory
// (the FP64 grid for FP64 outputs, its FP32 copy for FP32 outputs);
// arithmetic is FP64 in both cases.  MODE (VGX_EXTRAP_*) is a template
// parameter so that the default ERROR kernel carries no code of the other
// modes.
//
// A wave takes 64 consecutive queries at a time, in three phases.
//  1. One lane per query: subgrid, cells, the x and Q^2 weights of the
//     stencil (cubic Hermite; the bilinear rule as weights (1 - t, t, 0, 0))
//     and the offset of its first node, into the query's LDS slot.
//  2. ceil(nf / V) lanes per query, V = 16 / sizeof(ValT) flavours per lane
//     (2 FP64, 4 FP32): each lane gathers its flavours of the stencil's 16
//     nodes, one 16-byte load per node, and sums w_rk = q_r c_k times the
//     node values in row-major order (the bilinear stencil as 16 terms of
//     which 12 have zero weight and add exactly nothing).  The lanes of a
//     query read a node's nf contiguous values in one instruction, a
//     coalesced run of one to three 64-byte lines, 10 (FP64) or 21 (FP32)
//     queries per instruction.  One query per lane, reading whole stencil
//     rows per lane, made the L1 look up a line per lane and per 16 bytes
//     (88 lookups per query in FP64, with the texture addresser 98 % busy and
//     stalled by the L1 two thirds of the time); this layout measured 2.1x
//     (FP64) and 1.27x (FP32) faster.
//  3. One lane per query: the sums from the slot, stored structure-of-arrays
//     (coalesced).
// 16 bytes of grid values at the alignment of one value
template <typename T>
using Vec16 = T __attribute__((ext_vector_type(16 / sizeof(T)), aligned(sizeof(T))));

template <typename OutT, typename ValT, int NF, int MODE>
__global__ __launch_bounds__(256) void k_pdf_interp(PdfKernelArgs g, int64_t n, const double* __restrict__ qx,
                                                     const double* __restrict__ qq2,
                                                     const double* __restrict__ kx, const double* __restrict__ klx,
                                                     const double* __restrict__ kq2, const double* __restrict__ klq2,
                                                     const ValT* __restrict__ vals, OutT* __restrict__ out,
                                                     unsigned long long* __restrict__ oor) {
  extern __shared__ double lds[];
  double* sx = lds;                 // [n_x]
  double* slx = sx + g.n_x;         // [n_x]
  const int nqt = g.q_off[g.n_sub];
  double* sq2 = slx + g.n_x;        // [nqt]
  double* slq2 = sq2 + nqt;         // [nqt]
  for (int k = threadIdx.x; k < g.n_x; k += blockDim.x) { sx[k] = kx[k]; slx[k] = klx[k]; }
  for (int k = threadIdx.x; k < nqt; k += blockDim.x) { sq2[k] = kq2[k]; slq2[k] = klq2[k]; }
  __syncthreads();

  const int nf = NF > 0 ? NF : g.n_flav;
  const int SL = pdf_slot_doubles(nf);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* slots = slq2 + nqt + (size_t)wv * 64 * SL;
  double* mine = slots + lane * SL;
  const int64_t RS = (int64_t)g.n_x * nf;  // row stride in values
  constexpr int VPL = 16 / sizeof(ValT);   // flavours per lane: one 16-byte load
  const int lpq = (nf + VPL - 1) / VPL;    // lanes per query
  const int qpg = 64 / lpq;                // queries per gather step
  const int sub = lane / lpq, f0 = VPL * (lane - sub * lpq);
  const int64_t n_tiles = (n + 63) >> 6;
  for (int64_t t = (int64_t)blockIdx.x * nw + wv; t < n_tiles; t += (int64_t)gridDim.x * nw) {
    // phase 1: one lane per query
    const int64_t q = (t << 6) + lane;
    int64_t tag = kTagNone;
    if (q < n) {
      double x = qx[q];
      double q2 = qq2[q];
      if constexpr (MODE == VGX_EXTRAP_FREEZE) {  // the nearest grid point
        if (x > 0.0 && q2 > 0.0 && isfinite(x) && isfinite(q2)) {
          x = fmin(fmax(x, sx[0]), sx[g.n_x - 1]);
          q2 = fmin(fmax(q2, g.q2_lo[0]), g.q2_hi[g.n_sub - 1]);
        }
      }
      int s = -1;
      for (int k = 0; k < g.n_sub; ++k) {
        const bool last = (k == g.n_sub - 1);
        if (q2 >= g.q2_lo[k] && (q2 < g.q2_hi[k] || (last && q2 <= g.q2_hi[k]))) s = k;
      }
      tag = kTagNaN;
      if (s < 0 || !(x >= sx[0] && x <= sx[g.n_x - 1])) {
        if constexpr (MODE == VGX_EXTRAP_CONTINUE) {  // k_pdf_continue writes these
          if (x > 0.0 && q2 > 0.0 && isfinite(x) && isfinite(q2) && x <= sx[g.n_x - 1]) tag = kTagSkip;
        }
        if (tag == kTagNaN) atomicAdd(oor, 1ull);
      } else {
        const int nq = g.nq[s];
        const double* lq = slq2 + g.q_off[s];
        const int i = find_cell(sx, g.n_x, x);
        const int j = find_cell(sq2 + g.q_off[s], nq, q2);
        const double a = log(x), b = log(q2);
        double cx[4], cq[4];
        const bool full = i >= 1 && i <= g.n_x - 3 && j >= 1 && j <= nq - 3;
        int i0 = i, j0 = j;
        if (full) {
          const double ha = slx[i + 1] - slx[i];
          const double hb = lq[j + 1] - lq[j];
          hermite_weights((a - slx[i]) / ha, ha / (slx[i] - slx[i - 1]), ha / (slx[i + 2] - slx[i + 1]), cx);
          hermite_weights((b - lq[j]) / hb, hb / (lq[j] - lq[j - 1]), hb / (lq[j + 2] - lq[j + 1]), cq);
          i0 = i - 1;
          j0 = j - 1;
        } else {
          const double ta = (a - slx[i]) / (slx[i + 1] - slx[i]);
          const double tb = (b - lq[j]) / (lq[j + 1] - lq[j]);
          cx[0] = 1.0 - ta; cx[1] = ta; cx[2] = 0.0; cx[3] = 0.0;
          cq[0] = 1.0 - tb; cq[1] = tb; cq[2] = 0.0; cq[3] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) { mine[k] = cx[k]; mine[4 + k] = cq[k]; }
        tag = 2 * (((int64_t)(g.q_off[s] + j0) * g.n_x + i0) * nf) + (full ? 1 : 0);
      }
    }
    mine[8] = __longlong_as_double(tag);
    wave_lds_sync();
    // phase 2: nf lanes per query
    for (int g0 = 0; g0 < 64; g0 += qpg) {
      const int ql = g0 + sub;
      if (sub < qpg && ql < 64) {
        double* sl = slots + ql * SL;
        const int64_t tg = __double_as_longlong(sl[8]);
        if (tg >= 0) {
          const ValT* V = vals + (tg >> 1) + f0;
          const bool full = tg & 1;
          double c[4], d[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) { c[k] = sl[k]; d[k] = sl[4 + k]; }
          // the bilinear stencil's weights vanish for r >= 2 or k >= 2; those
          // terms read nodes of its own cell (in bounds) and add exactly zero
          // (grid values are finite), so every query runs the same 16 terms
          const int64_t ro[4] = {0, RS, full ? 2 * RS : 0, full ? 3 * RS : RS};
          const int ko[4] = {0, nf, full ? 2 * nf : 0, full ? 3 * nf : nf};
          // flavours f0 .. f0 + VPL - 1 in one 16-byte load (where nf is not
          // a multiple of VPL the last lane also reads the next node's first
          // values, or the grid's zero tail: read, weighted and dropped)
          double acc[VPL];
#pragma unroll
          for (int u = 0; u < VPL; ++u) acc[u] = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const double w = d[r] * c[k];
              const Vec16<ValT> v = *(const Vec16<ValT>*)(V + ro[r] + ko[k]);
#pragma unroll
              for (int u = 0; u < VPL; ++u) acc[u] = fma(w, (double)v[u], acc[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < VPL; ++u)  // after this query's reads of its slot
            if (f0 + u < nf) sl[f0 + u] = acc[u];
        }
      }
    }
    wave_lds_sync();
    // phase 3: one lane per query
    if (tag >= 0) {
      for (int f = 0; f < nf; ++f) out[(int64_t)f * n + q] = (OutT)mine[f];
    } else if (tag == kTagNaN) {
      for (int f = 0; f < nf; ++f) out[(int64_t)f * n + q] = (OutT)NAN;
    }
    wave_lds_sync();  // the slots are refilled for the next 64 queries
  }
}

// Several members of a PDF set at the same points (the thesis's multi-member
// evaluation for FastKernel-type convolutions): blockIdx.y is the member, so
// a wave takes 64 consecutive points of one member and its stores are
// contiguous; a set of N_rep members at a few thousand points still fills the
// chip.  One (point, member) per lane, each lane reading its stencil rows as
// 16-byte loads, in the weights and summation order of k_pdf_interp.  This
// workload is small (a few thousand points per member, a couple of waves'
// worth of work per member for each CU), and there one query per lane,
// with its higher occupancy, measured 1.25x faster than the cooperative
// gathers of k_pdf_interp.  Outside the grid: NaN (counted once
// per point, by member 0), whatever the context's extrapolation mode.
template <typename OutT, typename ValT, int NF>
__global__ __launch_bounds__(256) void k_pdf_members(PdfKernelArgs g, int64_t n, int64_t member_stride,
                                                     const double* __restrict__ qx, const double* __restrict__ qq2,
                                                     const double* __restrict__ kx, const double* __restrict__ klx,
                                                     const double* __restrict__ kq2, const double* __restrict__ klq2,
                                                     const ValT* __restrict__ vals, OutT* __restrict__ out,
                                                     unsigned long long* __restrict__ oor) {
  constexpr int NFM = NF > 0 ? NF : VGX_MAX_FLAV;
  extern __shared__ double lds[];
  double* sx = lds;
  double* slx = sx + g.n_x;
  const int nqt = g.q_off[g.n_sub];
  double* sq2 = slx + g.n_x;
  double* slq2 = sq2 + nqt;
  for (int k = threadIdx.x; k < g.n_x; k += blockDim.x) { sx[k] = kx[k]; slx[k] = klx[k]; }
  for (int k = threadIdx.x; k < nqt; k += blockDim.x) { sq2[k] = kq2[k]; slq2[k] = klq2[k]; }
  __syncthreads();
  const int nf = NF > 0 ? NF : g.n_flav;
  const int m = blockIdx.y;
  const ValT* Vm = vals + (int64_t)m * member_stride;
  OutT* om = out + (int64_t)m * nf * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const double x = qx[q];
    const double q2 = qq2[q];
    int s = -1;
    for (int k = 0; k < g.n_sub; ++k) {
      const bool last = (k == g.n_sub - 1);
      if (q2 >= g.q2_lo[k] && (q2 < g.q2_hi[k] || (last && q2 <= g.q2_hi[k]))) s = k;
    }
    if (s < 0 || !(x >= sx[0] && x <= sx[g.n_x - 1])) {
      for (int f = 0; f < nf; ++f) om[(int64_t)f * n + q] = (OutT)NAN;
      if (m == 0) atomicAdd(oor, 1ull);
      continue;
    }
    const int nq = g.nq[s];
    const double* lq = slq2 + g.q_off[s];
    const int i = find_cell(sx, g.n_x, x);
    const int j = find_cell(sq2 + g.q_off[s], nq, q2);
    const double a = log(x), b = log(q2);
    const ValT* V = Vm + (int64_t)g.q_off[s] * g.n_x * nf;
    double acc[NFM];
#pragma unroll
    for (int f = 0; f < NFM; ++f) acc[f] = 0.0;
    if (i >= 1 && i <= g.n_x - 3 && j >= 1 && j <= nq - 3) {
      const double ha = slx[i + 1] - slx[i];
      const double hb = lq[j + 1] - lq[j];
      double cx[4], cq[4];
      hermite_weights((a - slx[i]) / ha, ha / (slx[i] - slx[i - 1]), ha / (slx[i + 2] - slx[i + 1]), cx);
      hermite_weights((b - lq[j]) / hb, hb / (lq[j] - lq[j - 1]), hb / (lq[j + 2] - lq[j + 1]), cq);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const ValT* row = V + ((int64_t)(j - 1 + r) * g.n_x + (i - 1)) * nf;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double w = cq[r] * cx[k];
          const ValT* node = row + k * nf;
#pragma unroll
          for (int f = 0; f < NFM; ++f)
            if (f < nf) acc[f] = fma(w, (double)node[f], acc[f]);
        }
      }
    } else {
      const double ta = (a - slx[i]) / (slx[i + 1] - slx[i]);
      const double tb = (b - lq[j]) / (lq[j + 1] - lq[j]);
      const double w[4] = {(1.0 - ta) * (1.0 - tb), ta * (1.0 - tb), (1.0 - ta) * tb, ta * tb};
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const ValT* row = V + ((int64_t)(j + r) * g.n_x + i) * nf;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const ValT* node = row + k * nf;
#pragma unroll
          for (int f = 0; f < NFM; ++f)
            if (f < nf) acc[f] = fma(w[2 * r + k], (double)node[f], acc[f]);
        }
      }
    }
#pragma unroll
    for (int f = 0; f < NFM; ++f)
      if (f < nf) om[(int64_t)f * n + q] = (OutT)acc[f];
  }
}

// Second pass of a CONTINUE-mode call: the queries outside the grid that
// k_pdf_interp skipped.  A separate kernel, because inlined into the
// interpolation loop the FP64 exp/log of the continuation raise its
// register count (their constants are hoisted out of the loop); the rescan
// reads 16 bytes per query.  Knots are read from global memory: few queries
// take this path.
template <typename OutT, typename ValT>
__global__ __launch_bounds__(256) void k_pdf_continue(PdfKernelArgs g, int64_t n, const double* __restrict__ qx,
                                                      const double* __restrict__ qq2, const double* __restrict__ kx,
                                                      const double* __restrict__ klx, const double* __restrict__ kq2,
                                                      const double* __restrict__ klq2, const ValT* __restrict__ vals,
                                                      OutT* __restrict__ out) {
  const double xlo = kx[0], xhi = kx[g.n_x - 1];
  const double qlo = g.q2_lo[0], qhi = g.q2_hi[g.n_sub - 1];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const double x = qx[q], q2 = qq2[q];
    const bool valid = x > 0.0 && q2 > 0.0 && isfinite(x) && isfinite(q2) && x <= xhi;
    if (!valid || (x >= xlo && q2 >= qlo && q2 <= qhi)) continue;
    int s = -1;
    for (int k = 0; k < g.n_sub; ++k) {
      const bool last = (k == g.n_sub - 1);
      if (q2 >= g.q2_lo[k] && (q2 < g.q2_hi[k] || (last && q2 <= g.q2_hi[k]))) s = k;
    }
    const int i = x >= xlo ? find_cell(kx, g.n_x, x) : -1;
    for (int f = 0; f < g.n_flav; ++f)
      out[(int64_t)f * n + q] = (OutT)continue_value(g, vals, kx, klx, kq2, klq2, g.n_flav, s, i, x, q2, f);
  }
}

// alpha_s(Q): log-cubic interpolation on the table's subgrids (thesis PDF
// chapter, alpha_s paragraphs): cubic Hermite in ln Q^2 with secant-average
// slopes on interior cells, linear on a subgrid's edge cells, the top value
// above the last knot.  Below the first knot: NaN (ERROR), the first value
// (FREEZE), or the low-x line rule in ln Q^2 through the two lowest knots
// (CONTINUE).  Non-positive or non-finite Q^2: NaN.
struct AlphasArgs {
  int n_sub;
  int nq[VGX_MAX_SUB];
  int off[VGX_MAX_SUB + 1];
  double q2_lo[VGX_MAX_SUB], q2_hi[VGX_MAX_SUB];
  double top;
  int mode;
};

__global__ __launch_bounds__(256) void k_alphas(AlphasArgs g, int64_t n, const double* __restrict__ qq2,
                                                const double* __restrict__ klq2, const double* __restrict__ kval,
                                                double* __restrict__ out) {
  extern __shared__ double lds[];
  const int nt = g.off[g.n_sub];
  double* sl = lds;        // ln Q^2 knots
  double* sv = lds + nt;   // values
  for (int k = threadIdx.x; k < nt; k += blockDim.x) { sl[k] = klq2[k]; sv[k] = kval[k]; }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const double q2 = qq2[q];
    if (!(q2 > 0.0 && isfinite(q2))) { out[q] = (double)NAN; continue; }
    if (q2 > g.q2_hi[g.n_sub - 1]) { out[q] = g.top; continue; }
    if (q2 < g.q2_lo[0]) {
      out[q] = g.mode == VGX_EXTRAP_FREEZE     ? sv[0]
               : g.mode == VGX_EXTRAP_CONTINUE ? continue_line((log(q2) - sl[0]) / (sl[1] - sl[0]), sv[0], sv[1])
                                               : (double)NAN;
      continue;
    }
    int s = -1;
    for (int k = 0; k < g.n_sub; ++k) {
      const bool last = (k == g.n_sub - 1);
      if (q2 >= g.q2_lo[k] && (q2 < g.q2_hi[k] || (last && q2 <= g.q2_hi[k]))) s = k;
    }
    if (s < 0) { out[q] = (double)NAN; continue; }
    const double* b = sl + g.off[s];
    const double* v = sv + g.off[s];
    const int nq = g.nq[s];
    const double lb = log(q2);
    int lo = 0, hi = nq - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (b[mid] <= lb) lo = mid; else hi = mid;
    }
    const int j = lo;
    const double h = b[j + 1] - b[j];
    const double t = (lb - b[j]) / h;
    double r;
    if (j >= 1 && j <= nq - 3) {
      double c[4];
      hermite_weights(t, h / (b[j] - b[j - 1]), h / (b[j + 2] - b[j + 1]), c);
      r = c[0] * v[j - 1] + c[1] * v[j] + c[2] * v[j + 1] + c[3] * v[j + 2];
    } else {
      r = v[j] + t * (v[j + 1] - v[j]);
    }
    out[q] = r;
  }
}

}  // namespace vgx

using namespace vgx;

extern "C" vgx_status pdf_create(const vgx_pdf_desc* d, void* stream, vgx_pdf** out) {
  return pdf_create_set(d, 1, stream, out);
}

extern "C" vgx_status pdf_create_set(const vgx_pdf_desc* d, int32_t n_members, void* stream, vgx_pdf** out) {
  VGX_CHECK(d && out, "pdf_create: null argument");
  *out = nullptr;
  VGX_CHECK(n_members >= 1 && n_members <= 65535, "pdf_create_set: n_members %d out of 1..65535", n_members);
  VGX_CHECK(d->n_x >= 2 && d->n_sub >= 1 && d->n_sub <= VGX_MAX_SUB && d->n_flav >= 1 &&
                d->n_flav <= VGX_MAX_FLAV,
            "pdf_create: bad sizes n_x=%d n_sub=%d n_flav=%d", d->n_x, d->n_sub, d->n_flav);
  VGX_CHECK(d->x_knots && d->nq_per_sub && d->q2_knots && d->xf, "pdf_create: null array");
  for (int k = 0; k < d->n_x; ++k) {
    VGX_CHECK(d->x_knots[k] > 0.0 && (k == 0 || d->x_knots[k] > d->x_knots[k - 1]),
              "pdf_create: x knots must be positive and strictly ascending");
  }
  vgx_pdf* p = new vgx_pdf();
  p->n_x = d->n_x;
  p->n_sub = d->n_sub;
  p->n_flav = d->n_flav;
  p->n_members = n_members;
  p->fstride = d->n_flav;  // nodes stored densely (padding to 16 bytes measured slower)
  int tot = 0;
  for (int s = 0; s < d->n_sub; ++s) {
    if (d->nq_per_sub[s] < 2) { delete p; set_error("pdf_create: subgrid %d has < 2 knots", s); return VGX_EINVAL; }
    p->nq[s] = d->nq_per_sub[s];
    p->q_off[s] = tot;
    tot += d->nq_per_sub[s];
  }
  p->q_off[d->n_sub] = tot;
  if (pdf_interp_lds_bytes(p->n_x, tot, p->n_flav) > kMaxLds) {
    delete p;
    set_error("pdf_create: %d x knots and %d Q^2 knots exceed the interpolation kernel's LDS", d->n_x, tot);
    return VGX_EINVAL;
  }
  for (int s = 0; s < d->n_sub; ++s) {
    const double* q = d->q2_knots + p->q_off[s];
    for (int k = 0; k < p->nq[s]; ++k) {
      if (!(q[k] > 0.0) || (k > 0 && !(q[k] > q[k - 1]))) {
        delete p; set_error("pdf_create: Q^2 knots of subgrid %d must be positive, strictly ascending", s);
        return VGX_EINVAL;
      }
    }
    if (s > 0 && q[0] != d->q2_knots[p->q_off[s] - 1]) {
      delete p; set_error("pdf_create: subgrid %d must start at the previous subgrid's last knot", s);
      return VGX_EINVAL;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  hipGetDevice(&p->device);
  const size_t nmem = (size_t)tot * p->n_x * p->n_flav;  // values of one member
  const size_t nvals = nmem * (size_t)n_members;
  p->h_x = (double*)malloc(sizeof(double) * p->n_x);
  p->h_q2 = (double*)malloc(sizeof(double) * tot);
  double* lx = (double*)malloc(sizeof(double) * p->n_x);
  double* lq = (double*)malloc(sizeof(double) * tot);
  double* v = (double*)malloc(sizeof(double) * nvals);
  float* v32 = (float*)malloc(sizeof(float) * nvals);
  if (!p->h_x || !p->h_q2 || !lx || !lq || !v || !v32) {
    free(lx); free(lq); free(v); free(v32); pdf_destroy(p);
    set_error("pdf_create: host allocation failed");
    return VGX_ENOMEM;
  }
  for (int k = 0; k < p->n_x; ++k) { p->h_x[k] = d->x_knots[k]; lx[k] = log(d->x_knots[k]); }
  for (int k = 0; k < tot; ++k) { p->h_q2[k] = d->q2_knots[k]; lq[k] = log(d->q2_knots[k]); }
  // re-layout each member's [sub][flav][iq][ix] -> [member][iq_total][ix][flav]
  size_t src = 0;
  for (int m = 0; m < n_members; ++m)
    for (int s = 0; s < p->n_sub; ++s)
      for (int f = 0; f < p->n_flav; ++f)
        for (int iq = 0; iq < p->nq[s]; ++iq)
          for (int ix = 0; ix < p->n_x; ++ix, ++src) {
            const size_t dst = nmem * m + ((size_t)(p->q_off[s] + iq) * p->n_x + ix) * p->n_flav + f;
            v[dst] = d->xf[src];
            v32[dst] = (float)d->xf[src];
          }
  // finite values (in FP32 too): the interpolation kernels pad the bilinear
  // stencil with zero-weight terms, which are exact no-ops only on finite values
  for (size_t k = 0; k < nvals; ++k) {
    if (!(fabs(v[k]) <= (double)FLT_MAX)) {
      free(lx); free(lq); free(v); free(v32); pdf_destroy(p);
      set_error("pdf_create: grid value %zu is not finite (or beyond the FP32 range)", k);
      return VGX_EINVAL;
    }
  }
  vgx_status st_ = VGX_OK;
  do {
    if ((st_ = dev_alloc((void**)&p->x, sizeof(double) * p->n_x)) != VGX_OK) break;
    if ((st_ = dev_alloc((void**)&p->lx, sizeof(double) * p->n_x)) != VGX_OK) break;
    if ((st_ = dev_alloc((void**)&p->q2, sizeof(double) * tot)) != VGX_OK) break;
    if ((st_ = dev_alloc((void**)&p->lq2, sizeof(double) * tot)) != VGX_OK) break;
    // 16 bytes of zero tail: the interpolation kernel reads a node's values
    // 16 bytes at a time, up to 12 bytes beyond the last node
    if ((st_ = dev_alloc((void**)&p->v64, sizeof(double) * (nvals + 2))) != VGX_OK) break;
    if ((st_ = dev_alloc((void**)&p->v32, sizeof(float) * (nvals + 4))) != VGX_OK) break;
    if ((st_ = dev_alloc((void**)&p->oor, sizeof(unsigned long long))) != VGX_OK) break;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(p->x, p->h_x, sizeof(double) * p->n_x, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->lx, lx, sizeof(double) * p->n_x, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->q2, p->h_q2, sizeof(double) * tot, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->lq2, lq, sizeof(double) * tot, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->v64, v, sizeof(double) * nvals, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(p->v64 + nvals, 0, 2 * sizeof(double), st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->v32, v32, sizeof(float) * nvals, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(p->v32 + nvals, 0, 4 * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(p->oor, 0, sizeof(unsigned long long), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) st_ = hip_fail(e, "pdf_create copies", __FILE__, __LINE__);
  } while (0);
  free(lx); free(lq); free(v); free(v32);
  if (st_ != VGX_OK) { pdf_destroy(p); return st_; }
  *out = p;
  return VGX_OK;
}

template <int M>
static void launch_interp(const vgx_pdf* p, const PdfKernelArgs& g, dim3 grid, int block, size_t lds, hipStream_t st,
                          int64_t n, const double* x_dev, const double* q2_dev, int32_t out_dtype, void* out_dev) {
  const bool f11 = p->n_flav == 11;
  if (out_dtype == VGX_F64) {
    auto k = f11 ? k_pdf_interp<double, double, 11, M> : k_pdf_interp<double, double, 0, M>;
    hipLaunchKernelGGL(k, grid, dim3(block), lds, st, g, n, x_dev, q2_dev, p->x, p->lx, p->q2, p->lq2,
                       p->v64, (double*)out_dev, p->oor);
  } else {
    auto k = f11 ? k_pdf_interp<float, float, 11, M> : k_pdf_interp<float, float, 0, M>;
    hipLaunchKernelGGL(k, grid, dim3(block), lds, st, g, n, x_dev, q2_dev, p->x, p->lx, p->q2, p->lq2,
                       p->v32, (float*)out_dev, p->oor);
  }
}

extern "C" vgx_status pdf_interp(const vgx_pdf* p, int64_t n, const double* x_dev, const double* q2_dev,
                                 int32_t out_dtype, void* out_dev, void* stream) {
  VGX_CHECK(p, "pdf_interp: null context");
  VGX_CHECK(n >= 0, "pdf_interp: n < 0");
  VGX_CHECK(out_dtype == VGX_F64 || out_dtype == VGX_F32, "pdf_interp: bad out_dtype %d", out_dtype);
  if (n == 0) return VGX_OK;
  VGX_CHECK(x_dev && q2_dev && out_dev, "pdf_interp: null device pointer");
  PdfKernelArgs g{};
  g.n_x = p->n_x; g.n_sub = p->n_sub; g.n_flav = p->n_flav;
  for (int s = 0; s < p->n_sub; ++s) {
    g.nq[s] = p->nq[s];
    g.q_off[s] = p->q_off[s];
    g.q2_lo[s] = p->h_q2[p->q_off[s]];
    g.q2_hi[s] = p->h_q2[p->q_off[s] + p->nq[s] - 1];
  }
  g.q_off[p->n_sub] = p->q_off[p->n_sub];
  const int block = kInterpBlock;
  const int64_t want = (n + block - 1) / block;
  const int grid = (int)(want < (int64_t)device_cus() * 8 ? want : (int64_t)device_cus() * 8);
  const size_t lds = pdf_interp_lds_bytes(p->n_x, p->q_off[p->n_sub], p->n_flav);
  hipStream_t st = (hipStream_t)stream;
  auto launch = [&](auto mode_tag) {
    constexpr int M = decltype(mode_tag)::value;
    launch_interp<M>(p, g, dim3(grid), block, lds, st, n, x_dev, q2_dev, out_dtype, out_dev);
  };
  if (p->extrap == VGX_EXTRAP_FREEZE) launch(std::integral_constant<int, VGX_EXTRAP_FREEZE>{});
  else if (p->extrap == VGX_EXTRAP_CONTINUE) launch(std::integral_constant<int, VGX_EXTRAP_CONTINUE>{});
  else launch(std::integral_constant<int, VGX_EXTRAP_ERROR>{});
  VGX_HIP(hipGetLastError());
  if (p->extrap == VGX_EXTRAP_CONTINUE) {
    if (out_dtype == VGX_F64)
      hipLaunchKernelGGL((k_pdf_continue<double, double>), dim3(grid), dim3(block), 0, st, g, n, x_dev, q2_dev, p->x,
                         p->lx, p->q2, p->lq2, p->v64, (double*)out_dev);
    else
      hipLaunchKernelGGL((k_pdf_continue<float, float>), dim3(grid), dim3(block), 0, st, g, n, x_dev, q2_dev, p->x,
                         p->lx, p->q2, p->lq2, p->v32, (float*)out_dev);
    VGX_HIP(hipGetLastError());
  }
  return VGX_OK;
}

extern "C" vgx_status pdf_interp_members(const vgx_pdf* p, int64_t n, const double* x_dev, const double* q2_dev,
                                         int32_t out_dtype, void* out_dev, void* stream) {
  VGX_CHECK(p, "pdf_interp_members: null context");
  VGX_CHECK(n >= 0, "pdf_interp_members: n < 0");
  VGX_CHECK(out_dtype == VGX_F64 || out_dtype == VGX_F32, "pdf_interp_members: bad out_dtype %d", out_dtype);
  if (n == 0) return VGX_OK;
  VGX_CHECK(x_dev && q2_dev && out_dev, "pdf_interp_members: null device pointer");
  PdfKernelArgs g{};
  g.n_x = p->n_x; g.n_sub = p->n_sub; g.n_flav = p->n_flav;
  for (int s = 0; s < p->n_sub; ++s) {
    g.nq[s] = p->nq[s];
    g.q_off[s] = p->q_off[s];
    g.q2_lo[s] = p->h_q2[p->q_off[s]];
    g.q2_hi[s] = p->h_q2[p->q_off[s] + p->nq[s] - 1];
  }
  g.q_off[p->n_sub] = p->q_off[p->n_sub];
  const int64_t stride = (int64_t)p->q_off[p->n_sub] * p->n_x * p->n_flav;
  const int block = 256;
  // blocks per member: enough to cover the points, the chip filled across members
  const int64_t want = (n + block - 1) / block;
  int64_t cap = (int64_t)device_cus() * 8 / p->n_members;
  cap = cap < 1 ? 1 : cap;
  const dim3 grid((unsigned)(want < cap ? want : cap), (unsigned)p->n_members);
  const size_t lds = sizeof(double) * (2 * (size_t)p->n_x + 2 * (size_t)p->q_off[p->n_sub]);
  hipStream_t st = (hipStream_t)stream;
  const bool f11 = p->n_flav == 11;
  if (out_dtype == VGX_F64) {
    if (f11)
      hipLaunchKernelGGL((k_pdf_members<double, double, 11>), grid, dim3(block), lds, st, g, n, stride, x_dev, q2_dev,
                         p->x, p->lx, p->q2, p->lq2, p->v64, (double*)out_dev, p->oor);
    else
      hipLaunchKernelGGL((k_pdf_members<double, double, 0>), grid, dim3(block), lds, st, g, n, stride, x_dev, q2_dev,
                         p->x, p->lx, p->q2, p->lq2, p->v64, (double*)out_dev, p->oor);
  } else {
    if (f11)
      hipLaunchKernelGGL((k_pdf_members<float, float, 11>), grid, dim3(block), lds, st, g, n, stride, x_dev, q2_dev,
                         p->x, p->lx, p->q2, p->lq2, p->v32, (float*)out_dev, p->oor);
    else
      hipLaunchKernelGGL((k_pdf_members<float, float, 0>), grid, dim3(block), lds, st, g, n, stride, x_dev, q2_dev,
                         p->x, p->lx, p->q2, p->lq2, p->v32, (float*)out_dev, p->oor);
  }
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

extern "C" vgx_status pdf_shape(const vgx_pdf* p, int32_t* n_flav, int32_t* n_members) {
  VGX_CHECK(p, "pdf_shape: null context");
  if (n_flav) *n_flav = p->n_flav;
  if (n_members) *n_members = p->n_members;
  return VGX_OK;
}

extern "C" vgx_status pdf_out_of_range(vgx_pdf* p, void* stream, int64_t* count) {
  VGX_CHECK(p && count, "pdf_out_of_range: null argument");
  unsigned long long c = 0;
  hipStream_t st = (hipStream_t)stream;
  VGX_HIP(hipMemcpyAsync(&c, p->oor, sizeof(c), hipMemcpyDeviceToHost, st));
  VGX_HIP(hipStreamSynchronize(st));
  VGX_HIP(hipMemsetAsync(p->oor, 0, sizeof(c), st));
  VGX_HIP(hipStreamSynchronize(st));
  *count = (int64_t)c;
  return c ? VGX_ERANGE : VGX_OK;
}

extern "C" vgx_status pdf_set_extrapolation(vgx_pdf* p, int32_t mode) {
  VGX_CHECK(p, "pdf_set_extrapolation: null context");
  VGX_CHECK(mode == VGX_EXTRAP_ERROR || mode == VGX_EXTRAP_FREEZE || mode == VGX_EXTRAP_CONTINUE,
            "pdf_set_extrapolation: bad mode %d", mode);
  VGX_CHECK(mode != VGX_EXTRAP_CONTINUE || (p->n_x >= 2 && p->nq[0] >= 2),
            "pdf_set_extrapolation: continuation needs two x knots and two Q^2 knots in the lowest subgrid");
  p->extrap = mode;
  return VGX_OK;
}

extern "C" vgx_status pdf_bounds(const vgx_pdf* p, double* xmin, double* xmax, double* q2min, double* q2max) {
  VGX_CHECK(p, "pdf_bounds: null context");
  if (xmin) *xmin = p->h_x[0];
  if (xmax) *xmax = p->h_x[p->n_x - 1];
  if (q2min) *q2min = p->h_q2[0];
  if (q2max) *q2max = p->h_q2[p->q_off[p->n_sub] - 1];
  return VGX_OK;
}

extern "C" void pdf_destroy(vgx_pdf* p) {
  if (!p) return;
  hipFree(p->x); hipFree(p->lx); hipFree(p->q2); hipFree(p->lq2);
  hipFree(p->v64); hipFree(p->v32); hipFree(p->oor);
  hipFree(p->a_lq2); hipFree(p->a_val);
  free(p->h_x); free(p->h_q2); free(p->h_aq2); free(p->h_aval);
  delete p;
}

extern "C" vgx_status pdf_set_alphas(vgx_pdf* p, int32_t n, const double* q2_knots, const double* alphas,
                                     void* stream) {
  VGX_CHECK(p && q2_knots && alphas, "pdf_set_alphas: null argument");
  VGX_CHECK(n >= 2, "pdf_set_alphas: need at least 2 knots");
  // subgrids: a knot equal to the previous one starts a new subgrid
  int ns = 0, start = 0;
  int nq[VGX_MAX_SUB], off[VGX_MAX_SUB + 1];
  for (int k = 0; k < n; ++k) {
    VGX_CHECK(q2_knots[k] > 0.0 && isfinite(alphas[k]), "pdf_set_alphas: knots must be > 0, values finite");
    if (k > 0) {
      VGX_CHECK(q2_knots[k] >= q2_knots[k - 1], "pdf_set_alphas: knots must be ascending");
      if (q2_knots[k] == q2_knots[k - 1]) {
        VGX_CHECK(ns < VGX_MAX_SUB - 1, "pdf_set_alphas: more than %d subgrids", VGX_MAX_SUB);
        VGX_CHECK(k - start >= 2, "pdf_set_alphas: subgrid %d has < 2 knots", ns);
        off[ns] = start; nq[ns] = k - start; ++ns; start = k;
      }
    }
  }
  VGX_CHECK(n - start >= 2, "pdf_set_alphas: subgrid %d has < 2 knots", ns);
  off[ns] = start; nq[ns] = n - start; ++ns; off[ns] = n;
  double* hq = (double*)malloc(sizeof(double) * n);
  double* hv = (double*)malloc(sizeof(double) * n);
  double* lq = (double*)malloc(sizeof(double) * n);
  if (!hq || !hv || !lq) { free(hq); free(hv); free(lq); set_error("pdf_set_alphas: host allocation failed"); return VGX_ENOMEM; }
  for (int k = 0; k < n; ++k) { hq[k] = q2_knots[k]; hv[k] = alphas[k]; lq[k] = log(q2_knots[k]); }
  double *dl = nullptr, *dv = nullptr;
  vgx_status s = dev_alloc((void**)&dl, sizeof(double) * n);
  if (s == VGX_OK) s = dev_alloc((void**)&dv, sizeof(double) * n);
  if (s == VGX_OK) {
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(dl, lq, sizeof(double) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dv, hv, sizeof(double) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail(e, "pdf_set_alphas copies", __FILE__, __LINE__);
  }
  free(lq);
  if (s != VGX_OK) { hipFree(dl); hipFree(dv); free(hq); free(hv); return s; }
  hipFree(p->a_lq2); hipFree(p->a_val); free(p->h_aq2); free(p->h_aval);
  p->a_lq2 = dl; p->a_val = dv; p->h_aq2 = hq; p->h_aval = hv;
  p->a_nsub = ns;
  for (int k = 0; k < ns; ++k) { p->a_nq[k] = nq[k]; p->a_off[k] = off[k]; }
  p->a_off[ns] = n;
  return VGX_OK;
}

extern "C" vgx_status pdf_alphas(const vgx_pdf* p, int64_t n, const double* q2_dev, double* out_dev, void* stream) {
  VGX_CHECK(p, "pdf_alphas: null context");
  VGX_CHECK(n >= 0, "pdf_alphas: n < 0");
  if (n == 0) return VGX_OK;
  VGX_CHECK(p->a_nsub > 0, "pdf_alphas: no alpha_s table (pdf_set_alphas)");
  VGX_CHECK(q2_dev && out_dev, "pdf_alphas: null device pointer");
  AlphasArgs g{};
  g.n_sub = p->a_nsub;
  for (int s = 0; s < p->a_nsub; ++s) {
    g.nq[s] = p->a_nq[s];
    g.off[s] = p->a_off[s];
    g.q2_lo[s] = p->h_aq2[p->a_off[s]];
    g.q2_hi[s] = p->h_aq2[p->a_off[s] + p->a_nq[s] - 1];
  }
  g.off[p->a_nsub] = p->a_off[p->a_nsub];
  g.top = p->h_aval[p->a_off[p->a_nsub] - 1];
  g.mode = p->extrap;
  const int block = 256;
  const int64_t want = (n + block - 1) / block;
  const int grid = (int)(want < (int64_t)device_cus() * 8 ? want : (int64_t)device_cus() * 8);
  const size_t lds = sizeof(double) * 2 * (size_t)p->a_off[p->a_nsub];
  hipLaunchKernelGGL(k_alphas, dim3(grid), dim3(block), lds, (hipStream_t)stream, g, n, q2_dev, p->a_lq2, p->a_val,
                     out_dev);
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}
