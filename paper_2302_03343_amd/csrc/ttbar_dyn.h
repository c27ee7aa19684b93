// LO pp -> t tbar with the factorisation and renormalisation scale set per
// event, mu^2 = s_hat/4, and the running coupling alpha_s(mu) from the PDF
// set's alpha_s table (the fixed-scale integrand is in ttbar.h; kinematics
// and matrix elements are the same).
//
// Thesis, PDF chapter: xf(x, Q^2) by log-bicubic interpolation at any
// (x, Q^2), alpha_s(Q) by log-cubic interpolation on the table's knots.
// Here every event reads its own 4 x 4 stencil in (ln x, ln Q^2): the Q^2
// rows that the events' scales can reach, [m_t^2, s/4] plus the stencil
// margins, are staged in LDS as FP32 [row][node][12] (11 flavours and a pad:
// three 16-byte reads per row and node), the nodes of each row grouped by
// residue mod 4 as in pdf_rows.h.  Both axes use the same window rule: the
// full stencil with cubic Hermite weights (secant slopes) where both axes
// have their four knots, else bilinear on the cell corners written as the
// same 4 x 4 window with zero weights.  alpha_s: 4-knot cubic Hermite in
// ln Q^2 on its subgrid (linear on the edge cells), from an LDS copy.
#pragma once

#include "common.h"
#include "pdf_rows.h"

namespace vgx {

constexpr int TD_MAX_ROWS = 40;   // staged Q^2 rows
constexpr int TD_MAX_ALPHAS = 64; // knots of the alpha_s subgrid

struct TTDynConst {
  double L0;          // ln(1/tau0)
  double lns4;        // ln(s/4): ln mu^2 = ln(s/4) - ln(1/tau)
  float pref;         // 2 conv / (32 pi s)
  const float* v32;   // device [iq][ix][fstride] FP32 grid
  int fstride;
  const double* lx;   // device ln x knots
  int n_x, ix0, nxs;  // x knots; first staged node; staged nodes
  const double* lq2;  // device ln Q^2 knots of the subgrid holding the scales
  int q_glob;         // global knot index of the subgrid's first knot
  int nq;             // knots in that subgrid
  int r0, R;          // staged rows r0 .. r0 + R - 1 (subgrid-local)
  const double* a_lq2;// device ln Q^2 knots of the alpha_s subgrid
  const double* a_val;// device alpha_s values there
  int a_nq;           // knots in the alpha_s subgrid
  // cell guesses for knots uniform in ln x / ln Q^2 (set on the host)
  float a0, inv_da;   // first staged ln x, 1 / spacing
  int x_uniform;
  float b0, inv_db;   // first staged ln Q^2, 1 / spacing
  int q_uniform;
};

// LDS footprint in floats: node values [R][4][nxs/4 rounded up][12], ln x
// knots (padded to 4) and a float4 per x cell, ln Q^2 knots of the rows
// (padded to 4) and a float4 per row cell, the alpha_s knots and values.
__host__ __device__ inline int ttdyn_lds_floats(int nxs, int R, int a_nq) {
  return R * ((nxs + 3) & ~3) * 12 + ((nxs + 3) & ~3) + 4 * nxs + ((R + 3) & ~3) + 4 * R + 2 * a_nq;
}


// cell k with s[k] <= a < s[k+1] in a staged knot list of length n, clamped
// to [0, n - 2] (binary search)
__device__ __forceinline__ int knot_cell(const float* s, int n, float a) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s[mid] <= a) lo = mid; else hi = mid;
  }
  return lo;
}

// Hermite weights (secant-average slopes) of the nodes k-1..k+2 at fraction t
// of cell k, rm = h_k/h_{k-1}, rp = h_k/h_{k+1}
__device__ __forceinline__ void herm4(float t, float rm, float rp, float (&c)[4]) {
  const float t2 = t * t, t3 = t2 * t;
  const float h00 = 2.f * t3 - 3.f * t2 + 1.f, h10 = t3 - 2.f * t2 + t;
  const float h01 = -2.f * t3 + 3.f * t2, h11 = t3 - t2;
  c[0] = -0.5f * h10 * rm;
  c[1] = h00 - 0.5f * h10 + 0.5f * h10 * rm - 0.5f * h11;
  c[2] = h01 + 0.5f * h10 - 0.5f * h11 * rp + 0.5f * h11;
  c[3] = 0.5f * h11 * rp;
}

// linear weights (1 - t, t) at window positions pos, pos + 1
__device__ __forceinline__ void lin4(float t, int pos, float (&c)[4]) {
  const float u = 1.f - t;
  c[0] = pos == 0 ? u : 0.f;
  c[1] = pos == 1 ? u : (pos == 0 ? t : 0.f);
  c[2] = pos == 2 ? u : (pos == 1 ? t : 0.f);
  c[3] = pos == 2 ? t : 0.f;
}

struct TTbarDyn {
  static constexpr bool kStage = true;
  static constexpr int kMinWaves = 5;
  TTDynConst c;
  const float4* F;  // LDS [R][4][nq4][3] float4
  int nq4;
  float* sa;        // ln x knots [nxs]
  const float4* cwa;// per x cell (knot_cell_data)
  float* sb;        // ln Q^2 knots of the staged rows [R]
  const float4* cwb;// per row cell
  float* sal;       // ln Q^2 knots of the alpha_s subgrid [a_nq]
  float* sav;       // alpha_s values [a_nq]

  // the tables' places in an LDS block of ttdyn_lds_floats floats
  __device__ void layout(float* lds) {
    const int nxs = c.nxs, R = c.R;
    nq4 = (nxs + 3) >> 2;
    F = (const float4*)lds;
    sa = lds + R * nq4 * 4 * 12;
    cwa = (const float4*)(sa + ((nxs + 3) & ~3));
    sb = (float*)(cwa + nxs);
    cwb = (const float4*)(sb + ((R + 3) & ~3));
    sal = (float*)(cwb + R);
    sav = sal + c.a_nq;
  }

  // layout and fill the tables (every thread of the workgroup)
  __device__ void stage(float* lds) {
    layout(lds);
    const int nxs = c.nxs, R = c.R;
    float* Fs = lds;
    const int plane = nq4 * 4 * 12;  // floats per staged row
    float4* wa = const_cast<float4*>(cwa);
    float4* wb = const_cast<float4*>(cwb);
    const int tot = R * plane;
    for (int k = threadIdx.x; k < tot; k += blockDim.x) {
      const int f = k % 12;
      const int pos = (k / 12) % (nq4 * 4);  // (n mod 4) nq4 + n / 4
      const int r = k / plane;
      const int n = (pos % nq4) * 4 + pos / nq4;
      Fs[k] = (f < TT_NF && n < nxs)
                  ? c.v32[((size_t)(c.q_glob + c.r0 + r) * c.n_x + c.ix0 + n) * c.fstride + f]
                  : 0.0f;
    }
    const double* lx = c.lx + c.ix0;
    for (int k = threadIdx.x; k < nxs; k += blockDim.x) {
      sa[k] = (float)lx[k];
      wa[k] = knot_cell_data(lx, nxs, k);
    }
    const double* lb = c.lq2 + c.r0;
    for (int k = threadIdx.x; k < R; k += blockDim.x) {
      sb[k] = (float)lb[k];
      wb[k] = knot_cell_data(lb, R, k);
    }
    for (int k = threadIdx.x; k < c.a_nq; k += blockDim.x) {
      sal[k] = (float)c.a_lq2[k];
      sav[k] = (float)c.a_val[k];
    }
  }

  // x window of ln x = a: base node, Hermite and linear weights, full flag
  __device__ __forceinline__ void xwin(float a, int& base, float (&wh)[4], float (&wl)[4], bool& full) const {
    const int nx = c.nxs;
    const int klo = c.ix0 > 0 ? 1 : 0;
    int i = c.x_uniform ? uniform_knot_cell(sa, nx, a, c.a0, c.inv_da) : knot_cell(sa, nx, a);
    i = i < klo ? klo : i;
    const float4 q = cwa[i];
    const float t = (a - q.x) * q.y;
    full = i + c.ix0 >= 1 && i <= nx - 3;
    base = i - 1 < 0 ? 0 : (i - 1 > nx - 4 ? nx - 4 : i - 1);
    herm4(t, q.z, q.w, wh);
    lin4(t, i - base, wl);
  }

  // Q window of ln mu^2 = b in the staged rows: base row, weights, full flag
  __device__ __forceinline__ void qwin(float b, int& base, float (&wh)[4], float (&wl)[4], bool& full) const {
    const int R = c.R;
    const int jl = c.q_uniform ? uniform_knot_cell(sb, R, b, c.b0, c.inv_db) : knot_cell(sb, R, b);
    const int j = c.r0 + jl;  // subgrid-local cell
    const float4 q = cwb[jl];
    const float t = (b - q.x) * q.y;
    full = j >= 1 && j <= c.nq - 3;
    base = jl - 1 < 0 ? 0 : (jl - 1 > R - 4 ? R - 4 : jl - 1);
    herm4(t, q.z, q.w, wh);
    lin4(t, jl - base, wl);
  }

  // xf of all flavours at (ln x = a, the event's Q window)
  __device__ __forceinline__ void pdf_at(float a, int qb, bool qfull, const float (&qh)[4], const float (&ql)[4],
                                         float (&xf)[TT_NF]) const {
    int base;
    float wh[4], wl[4];
    bool xfull;
    xwin(a, base, wh, wl, xfull);
    const bool full = xfull && qfull;
    float w[4], q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[k] = full ? wh[k] : wl[k];
      q[k] = full ? qh[k] : ql[k];
    }
    // step k of the x window visits node 4 mb + k + 4 [k < r] (base = 4 mb + r)
    const int r = base & 3, mb = base >> 2;
    float cr[4];
    PdfRows::rotate(w, r, cr);
#pragma unroll
    for (int f = 0; f < TT_NF; ++f) xf[f] = 0.0f;
    // one Q row at a time (a rolled loop: 12 node reads in flight, not 48)
#pragma unroll 1
    for (int rr = 0; rr < 4; ++rr) {
      const float qr = rr == 0 ? q[0] : (rr == 1 ? q[1] : (rr == 2 ? q[2] : q[3]));
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int m = mb + (k < r ? 1 : 0);
        const float wk = cr[k] * qr;
        const float4* node = F + (size_t)((((qb + rr) * 4 + k) * nq4 + m) * 3);
        const float4 u0 = node[0], u1 = node[1], u2 = node[2];
        xf[0] = fmaf(wk, u0.x, xf[0]);
        xf[1] = fmaf(wk, u0.y, xf[1]);
        xf[2] = fmaf(wk, u0.z, xf[2]);
        xf[3] = fmaf(wk, u0.w, xf[3]);
        xf[4] = fmaf(wk, u1.x, xf[4]);
        xf[5] = fmaf(wk, u1.y, xf[5]);
        xf[6] = fmaf(wk, u1.z, xf[6]);
        xf[7] = fmaf(wk, u1.w, xf[7]);
        xf[8] = fmaf(wk, u2.x, xf[8]);
        xf[9] = fmaf(wk, u2.y, xf[9]);
        xf[10] = fmaf(wk, u2.z, xf[10]);
      }
    }
  }

  // alpha_s at ln mu^2 = b
  __device__ __forceinline__ float alphas(float b) const {
    const int n = c.a_nq;
    const int j = knot_cell(sal, n, b);
    const float hk = sal[j + 1] - sal[j];
    const float t = (b - sal[j]) / hk;
    if (j >= 1 && j <= n - 3) {
      float w[4];
      herm4(t, hk / (sal[j] - sal[j - 1]), hk / (sal[j + 2] - sal[j + 1]), w);
      return fmaf(w[0], sav[j - 1], fmaf(w[1], sav[j], fmaf(w[2], sav[j + 1], w[3] * sav[j + 2])));
    }
    return fmaf(t, sav[j + 1] - sav[j], sav[j]);
  }

  __device__ __forceinline__ double eval(const double (&x)[3]) const {
    const double v = x[0] * c.L0;                  // u1 L0
    const double ltau = (1.0 - x[0]) * c.L0;       // ln(1/tau)
    const double y = (x[1] - 0.5) * ltau;
    const float a1 = (float)(y - 0.5 * ltau);      // ln x1
    const float a2 = (float)(-y - 0.5 * ltau);     // ln x2
    const float b = (float)(c.lns4 - ltau);        // ln mu^2 = ln(s_hat/4)
    const float w3 = (float)(1.0 - x[2]);
    const float u3 = (float)x[2];
    const float vf = (float)v;
    const float rho = __expf(-vf);
    const float beta = __builtin_amdgcn_sqrtf(-expm1f(-vf));
    const float omb = rho * __builtin_amdgcn_rcpf(1.f + beta);
    const float tau1 = 0.5f * (omb + 2.f * beta * w3);
    const float tau2 = 0.5f * (omb + 2.f * beta * u3);
    const float t12 = tau1 * tau2;
    const float r12 = __builtin_amdgcn_rcpf(t12);
    const float ss = fmaf(tau1, tau1, tau2 * tau2);
    const float as = alphas(b);
    const float g2 = 4.f * 3.14159265358979f * as;
    const float g4 = g2 * g2;
    const float m_qq = g4 * (4.f / 9.f) * fmaf(0.5f, rho, ss);
    const float m_gg = g4 * fmaf(r12, 1.f / 6.f, -0.375f) * (ss + rho - 0.25f * rho * rho * r12);
    int qb;
    float qh[4], ql[4];
    bool qfull;
    qwin(b, qb, qh, ql, qfull);
    float f1[TT_NF], f2[TT_NF];
    pdf_at(a1, qb, qfull, qh, ql, f1);
    pdf_at(a2, qb, qfull, qh, ql, f2);
    const float lum_gg = f1[5] * f2[5];
    float lum_qq = 0.f;
#pragma unroll
    for (int q = 6; q < 11; ++q) lum_qq = fmaf(f1[q], f2[10 - q], fmaf(f1[10 - q], f2[q], lum_qq));
    const float inv_tau = __expf((float)ltau);
    const float jac = (float)(c.L0 * ltau);
    return (double)(c.pref * jac * beta * inv_tau * fmaf(lum_gg, m_gg, lum_qq * m_qq));
  }
};

}  // namespace vgx
