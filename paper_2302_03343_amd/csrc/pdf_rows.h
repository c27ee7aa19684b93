// PDF lookup at one fixed factorisation scale, served from LDS: the part of
// the fused hadronic integrands (t tbar, Drell-Yan) that reads the parton
// densities xf(x, mu^2) of all flavours at two momentum fractions per event.
//
// Thesis, PDF chapter: log-bicubic interpolation, cubic Hermite splines in
// (ln x, ln Q^2) on the four neighbouring knots of each axis, bilinear where
// that stencil is incomplete; subgrids separated at the flavour thresholds.
//
// Layout: the four Q^2 rows j-1..j+2 around mu^2 (two rows if the Q
// stencil is incomplete) are staged in LDS as FP32 [node][flav][row] (one
// 16-byte read per node and flavour), the nodes grouped by (node mod 4):
// step k of the 4-node stencil reads, in every lane, the stencil node
// congruent to k mod 4, so lanes whose cells lie close together read one
// address (a broadcast) and lanes further apart fall on distinct banks
// (consecutive groups of four nodes are 11 x 16 bytes apart, an odd multiple
// of 16 bytes).  Per event and per x the cubic Hermite (secant slopes) in
// ln x and then in ln Q^2 is evaluated for all 11 flavours, as a 4x4
// weighted sum w_rk = q_r c_k of the stencil (the same linear function as
// the Hermite-with-slopes formula).  Only nodes from two cells below the
// smallest reachable ln x are staged.  Flavour order: -5..-1, g, 1..5.
//
// Mode 1 ("contract") uses that the scale is fixed: the Q^2 direction is
// contracted once per workgroup into one table per x node (Hermite weights
// for full-stencil cells, linear weights for bilinear ones); the result is
// the same interpolant up to FP32 rounding order.
#pragma once

#include "common.h"
#include "pdf_internal.h"

namespace vgx {

constexpr int TT_NF = 11;
constexpr int TT_MAX_NX = 256;

struct PdfRowsConst {
  const float* v32; // device [iq][ix][fstride] FP32 grid
  int fstride;
  const double* lx; // device ln x knots
  int n_x;          // x knots of the grid
  int ix0;          // first staged x node: events never reach ln x below the
                    // smallest reachable momentum fraction, so nodes below
                    // its cell (less a margin of two cells) are not staged
  int nxs;          // staged x nodes, n_x - ix0
  int row0;         // global index of the first staged Q^2 row
  int n_rows;       // 4 (bicubic in Q) or 2 (bilinear in Q)
  int contract;     // 1: Q^2 direction contracted once per workgroup
  // set on the host from the knots (kernel arguments, so scalar registers):
  float qh[4];      // Q-row weights at mu^2: cubic Hermite on rows 0..3 (four rows), or linear on rows 0, 1
  float ql[4];      // linear Q weights on the cell (j, j + 1): the bilinear rule's rows
  float a0, inv_da; // cell guess for knots uniform in ln x: first staged ln x, 1 / spacing
  int uniform;      // 1 when the staged ln x knots are uniform to 1e-3 of a spacing
};

// LDS footprint in floats for nxs staged x nodes: node values, padded to a
// multiple of 4 nodes, [4][nxs/4][11][4 rows] (16-byte aligned float4 per
// node and flavour), ln x knots (padded to 4) and a float4 per cell.
__host__ __device__ inline int pdf_rows_lds_floats(int nxs) {
  return ((nxs + 3) & ~3) * 4 * TT_NF + ((nxs + 3) & ~3) + 4 * nxs;
}

// Cell k of a knot list s[0..n) (FP32) with s[k] <= a < s[k+1], clamped to
// [0, n - 2], for knots uniform to 1e-3 of a spacing (FP32 rounding of the
// logarithms adds about 1e-5 of a spacing): the guess from the spacing is the
// right cell or its neighbour, and one comparison with each end of the
// guessed cell settles it (the same cell as a binary search over s).
__device__ __forceinline__ int uniform_knot_cell(const float* s, int n, float a, float a0, float inv_d) {
  int i = (int)((a - a0) * inv_d);
  i = i < 0 ? 0 : (i > n - 2 ? n - 2 : i);
  const float lo = s[i], hi = s[i + 1];
  return i + (a >= hi && i < n - 2 ? 1 : 0) - (a < lo && i > 0 ? 1 : 0);
}

// Per cell k of a knot list (FP32 knots s): (s_k, 1/h_k, h_k/h_{k-1},
// h_k/h_{k+1}) with h_k = s_{k+1} - s_k, h_{-1} read as h_0 and 1/h past
// the last knot as 0: the Hermite window's inputs in one 16-byte read.
__device__ __forceinline__ float4 knot_cell_data(const double* l, int n, int k) {
  auto inv = [&](int m) { return m + 1 < n ? (float)(1.0 / (l[m + 1] - l[m])) : 0.0f; };
  const float hk = k + 1 < n ? (float)l[k + 1] - (float)l[k] : 0.0f;
  return make_float4((float)l[k], inv(k), hk * inv(k >= 1 ? k - 1 : 0), hk * inv(k + 1));
}

struct PdfRows {
  PdfRowsConst c;
  // LDS tables are indexed by the staged node k = ix - ix0
  const float4* F;  // LDS [4][nq4][11] float4: the (up to) four Q^2 rows of one node and flavour
  int nq4;          // staged nodes per residue class mod 4
  float* sa;        // LDS ln x knots [nxs]
  float4* cw;       // LDS per cell: knot_cell_data

  // the tables' places in an LDS block of pdf_rows_lds_floats(nxs) floats
  __device__ void layout(float* lds) {
    F = (const float4*)lds;
    nq4 = (c.nxs + 3) >> 2;
    sa = lds + nq4 * 4 * 4 * TT_NF;
    cw = (float4*)(sa + ((c.nxs + 3) & ~3));
  }

  // layout and fill the tables (every thread of the workgroup)
  __device__ void stage(float* lds) {
    layout(lds);
    float* Fs = lds;
    const int nxs = c.nxs;
    const int nr = c.n_rows;
    const int tot = nq4 * 4 * TT_NF * 4;
    const double* lx = c.lx + c.ix0;
    for (int k = threadIdx.x; k < tot; k += blockDim.x) {
      const int r = k & 3;
      const int f = (k >> 2) % TT_NF;
      const int pos = (k >> 2) / TT_NF;            // (n mod 4) nq4 + n / 4
      const int n = (pos % nq4) * 4 + pos / nq4;   // staged node
      Fs[k] = (r < nr && n < nxs) ? c.v32[((size_t)(c.row0 + r) * c.n_x + c.ix0 + n) * c.fstride + f] : 0.0f;
    }
    for (int k = threadIdx.x; k < nxs; k += blockDim.x) {
      sa[k] = (float)lx[k];
      cw[k] = knot_cell_data(lx, nxs, k);
    }
    if (c.contract) {
      // fixed scale: contract the Q^2 direction once.  P with the Hermite Q
      // weights (cells with the full stencil) and Pl with the linear ones
      // (bilinear cells), 12 floats (3 x float4) per node, nodes grouped by
      // residue mod 4 like F.  The node values occupy F; the tables are
      // built in registers first.
      __syncthreads();
      float pv[2][(TT_MAX_NX * 12 + 255) / 256];
      const int tot12 = nq4 * 4 * 12;
      int q = 0;
      for (int k = threadIdx.x; k < tot12; k += blockDim.x, ++q) {
        const int f = k % 12, pos = k / 12;
        const int n = (pos % nq4) * 4 + pos / nq4;
        float hp = 0.f, lp = 0.f;
        if (f < TT_NF && n < nxs) {
          const float4 v = F[node_off(n) + f];
          hp = fmaf(c.qh[0], v.x, fmaf(c.qh[1], v.y, fmaf(c.qh[2], v.z, c.qh[3] * v.w)));
          lp = fmaf(c.ql[0], v.x, fmaf(c.ql[1], v.y, fmaf(c.ql[2], v.z, c.ql[3] * v.w)));
        }
        pv[0][q] = hp;
        pv[1][q] = lp;
      }
      __syncthreads();
      float* P = lds;
      q = 0;
      for (int k = threadIdx.x; k < tot12; k += blockDim.x, ++q) {
        P[k] = pv[0][q];
        P[tot12 + k] = pv[1][q];
      }
    }
  }

  // float4 offset of staged node n in F
  __device__ __forceinline__ int node_off(int n) const { return ((n & 3) * nq4 + (n >> 2)) * TT_NF; }

  // staged cell k with sa[k] <= a < sa[k+1], clamped to [k_lo, nxs - 2];
  // k_lo = 1 when nodes below the staged range exist (never reached by
  // events: it only keeps the stencil's node k - 1 inside the table)
  __device__ __forceinline__ int cell(float a) const {
    const int nx = c.nxs;
    const int klo = c.ix0 > 0 ? 1 : 0;
    if (c.uniform) {
      const int i = uniform_knot_cell(sa, nx, a, c.a0, c.inv_da);
      return i < klo ? klo : i;
    }
    int lo = 0, hi = nx - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (sa[mid] <= a) lo = mid; else hi = mid;
    }
    return lo > klo ? lo : klo;
  }

  // Stencil window of the cell holding ln x = a: nodes base..base+3 with x
  // weights w.  full: both axes have their four knots, w is the cubic
  // Hermite (secant slopes); else the bilinear fallback, expressed as the
  // same 4-node window with weights (1 - t, t) on the cell's corners and
  // zeros elsewhere, so that every lane runs one code path.  Bilinear cells
  // lie at the grid's edges: a wave whose lanes all have the full stencil
  // (nearly every wave) skips the fallback's weights.
  __device__ __forceinline__ void window(float a, int& base, float (&w)[4], bool& full) const {
    const int nx = c.nxs;
    const int i = cell(a);
    const float4 q = cw[i];
    const float t = (a - q.x) * q.y;
    full = c.n_rows == 4 && i + c.ix0 >= 1 && i <= nx - 3;
    base = i - 1 < 0 ? 0 : (i - 1 > nx - 4 ? nx - 4 : i - 1);
    const float rm = q.z, rp = q.w;
    const float t2 = t * t, t3 = t2 * t;
    const float h00 = 2.f * t3 - 3.f * t2 + 1.f, h10 = t3 - 2.f * t2 + t;
    const float h01 = -2.f * t3 + 3.f * t2, h11 = t3 - t2;
    w[0] = -0.5f * h10 * rm;
    w[1] = h00 - 0.5f * h10 + 0.5f * h10 * rm - 0.5f * h11;
    w[2] = h01 + 0.5f * h10 - 0.5f * h11 * rp + 0.5f * h11;
    w[3] = 0.5f * h11 * rp;
    if (!__all(full)) {
      const int pos = i - base;  // 1 for the full stencil
      const float u = 1.f - t;
      w[0] = full ? w[0] : (pos == 0 ? u : 0.f);
      w[1] = full ? w[1] : (pos == 1 ? u : (pos == 0 ? t : 0.f));
      w[2] = full ? w[2] : (pos == 2 ? u : (pos == 1 ? t : 0.f));
      w[3] = full ? w[3] : (pos == 2 ? t : 0.f);
    }
  }

  // step k of a window starting at base visits node 4 mb + k + 4 [k < r]
  // (base = 4 mb + r), the window position (k - r) mod 4: the weights
  // rotated by r
  __device__ __forceinline__ static void rotate(const float (&w)[4], int r, float (&cr)[4]) {
    const bool o1 = r & 1, o2 = r & 2;
    const float d0 = o1 ? w[3] : w[0], d1 = o1 ? w[0] : w[1];
    const float d2 = o1 ? w[1] : w[2], d3 = o1 ? w[2] : w[3];
    cr[0] = o2 ? d2 : d0;
    cr[1] = o2 ? d3 : d1;
    cr[2] = o2 ? d0 : d2;
    cr[3] = o2 ? d1 : d3;
  }

  // xf of all flavours at ln x = a (a <= 0).
  __device__ __forceinline__ void pdf_at(float a, float (&xf)[TT_NF]) const {
    int base;
    float w[4];
    bool full;
    window(a, base, w, full);
    const int r = base & 3, mb = base >> 2;
    float cr[4];
    rotate(w, r, cr);
    if (c.contract) {
      // Hermite-in-Q table for full cells, linear-in-Q table otherwise
      const float4* T = F + (full ? 0 : nq4 * 4 * 3);
      float v[12];
#pragma unroll
      for (int f = 0; f < 12; ++f) v[f] = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4* node = T + (size_t)((k * nq4 + mb + (k < r ? 1 : 0)) * 3);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const float4 u = node[m];
          v[4 * m] = fmaf(cr[k], u.x, v[4 * m]);
          v[4 * m + 1] = fmaf(cr[k], u.y, v[4 * m + 1]);
          v[4 * m + 2] = fmaf(cr[k], u.z, v[4 * m + 2]);
          v[4 * m + 3] = fmaf(cr[k], u.w, v[4 * m + 3]);
        }
      }
#pragma unroll
      for (int f = 0; f < TT_NF; ++f) xf[f] = v[f];
      return;
    }
    // Q weights: Hermite for full cells, linear on the cell otherwise
    float q0 = c.qh[0], q1 = c.qh[1], q2 = c.qh[2], q3 = c.qh[3];
    if (!__all(full)) {
      q0 = full ? q0 : c.ql[0];
      q1 = full ? q1 : c.ql[1];
      q2 = full ? q2 : c.ql[2];
      q3 = full ? q3 : c.ql[3];
    }
#pragma unroll
    for (int f = 0; f < TT_NF; ++f) xf[f] = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float w0 = cr[k] * q0, w1 = cr[k] * q1, w2 = cr[k] * q2, w3 = cr[k] * q3;
      const float4* node = F + (size_t)((k * nq4 + mb + (k < r ? 1 : 0)) * TT_NF);
#pragma unroll
      for (int f = 0; f < TT_NF; ++f) {
        const float4 v = node[f];
        xf[f] = fmaf(w0, v.x, fmaf(w1, v.y, fmaf(w2, v.z, fmaf(w3, v.w, xf[f]))));
      }
    }
  }
};

}  // namespace vgx
