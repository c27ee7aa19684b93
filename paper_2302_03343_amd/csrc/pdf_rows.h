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
  const double* lq2;// device ln Q^2 knots (all subgrids)
  int n_x;          // x knots of the grid
  int ix0;          // first staged x node: events never reach ln x below the
                    // smallest reachable momentum fraction, so nodes below
                    // its cell (less a margin of two cells) are not staged
  int nxs;          // staged x nodes, n_x - ix0
  int row0;         // global index of the first staged Q^2 row
  int n_rows;       // 4 (bicubic in Q) or 2 (bilinear in Q)
  int j_local;      // cell index of mu^2 inside its subgrid
  int nq_sub;       // knots in that subgrid
  int q_off;        // global knot offset of the subgrid
  double lmu2;      // ln mu^2
  int contract;     // 1: Q^2 direction contracted once per workgroup
};

// LDS footprint in floats for nxs staged x nodes: node values, padded to a
// multiple of 4 nodes, [4][nxs/4][11][4 rows] (16-byte aligned float4 per
// node and flavour), ln x knots, inverse spacings, Q weights and the
// cell-guess constants.
__host__ __device__ inline int pdf_rows_lds_floats(int nxs) {
  return ((nxs + 3) & ~3) * 4 * TT_NF + 2 * nxs + 16;
}

struct PdfRows {
  PdfRowsConst c;
  // LDS tables are indexed by the staged node k = ix - ix0
  const float4* F;  // LDS [4][nq4][11] float4: the (up to) four Q^2 rows of one node and flavour
  int nq4;          // staged nodes per residue class mod 4
  float* sa;        // LDS ln x knots [nxs]
  float* sinv;      // LDS 1/(a_{k+1} - a_k) [nxs]
  float* qw;        // LDS [0..3] Q-row Hermite weights, [4] bilinear t_b, [5] a_0, [6] 1/da, [7] uniform flag,
                    // [8..11] linear Q-row weights of the bilinear fallback

  __device__ void stage(float* lds) {
    float* Fs = lds;
    F = (const float4*)lds;
    const int nxs = c.nxs;
    nq4 = (nxs + 3) >> 2;
    sa = Fs + nq4 * 4 * 4 * TT_NF;
    sinv = sa + nxs;
    qw = sinv + nxs;
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
      sinv[k] = k + 1 < nxs ? (float)(1.0 / (lx[k + 1] - lx[k])) : 0.0f;
    }
    if (threadIdx.x == 0) {
      // weights of the Q rows at mu^2 (FP64 setup, FP32 storage)
      const double* lq = c.lq2 + c.q_off;
      const int j = c.j_local;
      const double hb = lq[j + 1] - lq[j];
      const double t = (c.lmu2 - lq[j]) / hb;
      if (c.n_rows == 4) {
        const double rm = hb / (lq[j] - lq[j - 1]), rp = hb / (lq[j + 2] - lq[j + 1]);
        const double t2 = t * t, t3 = t2 * t;
        const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
        qw[0] = (float)(-0.5 * h10 * rm);
        qw[1] = (float)(h00 - 0.5 * h10 + 0.5 * h10 * rm - 0.5 * h11);
        qw[2] = (float)(h01 + 0.5 * h10 - 0.5 * h11 * rp + 0.5 * h11);
        qw[3] = (float)(0.5 * h11 * rp);
      } else {
        qw[0] = (float)(1.0 - t);
        qw[1] = (float)t;
        qw[2] = 0.0f;
        qw[3] = 0.0f;
      }
      qw[4] = (float)t;  // linear weight in ln Q^2 for the bilinear fallback
      // cell guess for knots uniform in ln x (checked here; else binary search)
      const int n = nxs;
      const double a0 = lx[0], da = (lx[n - 1] - lx[0]) / (n - 1);
      bool uni = true;
      for (int k = 0; k < n; ++k)
        if (fabs(lx[k] - (a0 + k * da)) > 1e-3 * da) uni = false;
      qw[5] = (float)a0;
      qw[6] = (float)(1.0 / da);
      qw[7] = uni ? 1.0f : 0.0f;
    }
    if (threadIdx.x == 0) {
      // linear Q weights on the cell (j, j+1) for the bilinear fallback: rows
      // 1, 2 of four staged rows, or 0, 1 of two
      const float tb = qw[4];
      const bool four = c.n_rows == 4;
      qw[8] = four ? 0.0f : 1.0f - tb;
      qw[9] = four ? 1.0f - tb : tb;
      qw[10] = four ? tb : 0.0f;
      qw[11] = 0.0f;
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
          hp = fmaf(qw[0], v.x, fmaf(qw[1], v.y, fmaf(qw[2], v.z, qw[3] * v.w)));
          lp = fmaf(qw[8], v.x, fmaf(qw[9], v.y, qw[10] * v.z));
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
    if (qw[7] != 0.0f) {
      // guess from the uniform spacing, then settle on the stored knots
      // (the same cell as a binary search over sa)
      int i = (int)((a - qw[5]) * qw[6]);
      i = i < klo ? klo : (i > nx - 2 ? nx - 2 : i);
      while (i > klo && a < sa[i]) --i;
      while (i < nx - 2 && a >= sa[i + 1]) ++i;
      return i;
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
  // zeros elsewhere, so that every lane runs one code path.
  __device__ __forceinline__ void window(float a, int& base, float (&w)[4], bool& full) const {
    const int nx = c.nxs;
    const int i = cell(a);
    const float t = (a - sa[i]) * sinv[i];
    full = c.n_rows == 4 && i + c.ix0 >= 1 && i <= nx - 3;
    base = i - 1 < 0 ? 0 : (i - 1 > nx - 4 ? nx - 4 : i - 1);
    const int pos = i - base;  // 1 for the full stencil
    const float hk = sa[i + 1] - sa[i];
    const float rm = hk * sinv[i >= 1 ? i - 1 : 0];
    const float rp = hk * sinv[i + 1];
    const float t2 = t * t, t3 = t2 * t;
    const float h00 = 2.f * t3 - 3.f * t2 + 1.f, h10 = t3 - 2.f * t2 + t;
    const float h01 = -2.f * t3 + 3.f * t2, h11 = t3 - t2;
    const float c0 = -0.5f * h10 * rm;
    const float c1 = h00 - 0.5f * h10 + 0.5f * h10 * rm - 0.5f * h11;
    const float c2 = h01 + 0.5f * h10 - 0.5f * h11 * rp + 0.5f * h11;
    const float c3 = 0.5f * h11 * rp;
    const float u = 1.f - t;
    w[0] = full ? c0 : (pos == 0 ? u : 0.f);
    w[1] = full ? c1 : (pos == 1 ? u : (pos == 0 ? t : 0.f));
    w[2] = full ? c2 : (pos == 2 ? u : (pos == 1 ? t : 0.f));
    w[3] = full ? c3 : (pos == 2 ? t : 0.f);
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
    const float q0 = full ? qw[0] : qw[8], q1 = full ? qw[1] : qw[9];
    const float q2 = full ? qw[2] : qw[10], q3 = full ? qw[3] : qw[11];
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
