// Fused LO s-channel single-top integrand, u dbar (c sbar) -> W* -> t bbar:
// FP32 arithmetic, kinematics set up in FP64, the PDF lookup served from
// LDS (PdfRows at the fixed scale mu^2 = m_t^2).
//
// Thesis: the LO single-top example (physics-examples section; q qbar ->
// t bbar the only diagram) and the master formula (MadFlow chapter).  The
// matrix element (W vertex (g/sqrt 2) gamma^mu P_L, diagonal CKM matrix,
// colour factor 1) is |M|^2 = (g^4/4) |P_W|^2 u_hat (u_hat - m_t^2), with
// -u_hat = (s_hat - m_t^2)(1 + cos)/2, cos between the quark and the top;
// dsigma/dcos = |M|^2 beta/(32 pi s_hat), beta = 1 - m_t^2/s_hat.  A quark
// from the second beam sees the top at pi - theta.
// Map of the unit cube: tau = tau0^(1-x1), tau0 = m_t^2/s, so that
// s_hat = m_t^2 e^v, v = x1 ln(1/tau0), and (rounding-safe, no cancellation)
//   s_hat - m_t^2 = m_t^2 expm1(v),  beta = -expm1(-v),
//   u_hat (u_hat - m_t^2) = A x3 (A x3 + m_t^2),  A = s_hat - m_t^2
// (A (1 - x3) (A (1 - x3) + m_t^2) for the quark from the second beam), and
//   F = 2 L0 ln(1/tau) conv g^4/(128 pi) beta/s_hat |P_W|^2
//       * sum_pairs [xq(x1) xq'(x2) K(x3) + xq'(x1) xq(x2) K(1 - x3)].
#pragma once

#include "common.h"
#include "pdf_rows.h"

namespace vgx {

struct STConst {
  double L0;        // ln(1/tau0)
  float mt2;        // m_t^2
  float mw2, mwg2;  // M_W^2, (M_W Gamma_W)^2
  float pref;       // 2 L0 conv g^4 / (128 pi)
  PdfRowsConst pdf; // PDF rows at mu^2 = m_t^2, staged from x >= tau0
};

struct SingleTop {
  static constexpr bool kStage = true;
  STConst c;
  PdfRows P;

  __device__ void stage(float* lds) {
    P.c = c.pdf;
    P.stage(lds);
  }
  __device__ void layout(float* lds) {
    P.c = c.pdf;
    P.layout(lds);
  }

  __device__ __forceinline__ double eval(const double (&x)[3]) const {
    const double v = x[0] * c.L0;                  // ln(s_hat/m_t^2)
    const double ltau = (1.0 - x[0]) * c.L0;       // ln(1/tau)
    const double y = (x[1] - 0.5) * ltau;
    const float a1 = (float)(y - 0.5 * ltau);      // ln x1
    const float a2 = (float)(-y - 0.5 * ltau);     // ln x2
    const float vf = (float)v;
    const float em = expm1f(vf);                   // s_hat/m_t^2 - 1
    const float A = c.mt2 * em;                    // s_hat - m_t^2
    const float shat = c.mt2 + A;
    const float beta = -expm1f(-vf);
    const float dw = shat - c.mw2;
    const float pw = __builtin_amdgcn_rcpf(fmaf(dw, dw, c.mwg2));
    const float Af = A * (float)x[2], Ab = A * (float)(1.0 - x[2]);
    const float kf = Af * (Af + c.mt2);            // quark from beam 1
    const float kb = Ab * (Ab + c.mt2);            // quark from beam 2
    float f1[TT_NF], f2[TT_NF];
    P.pdf_at(a1, f1);
    P.pdf_at(a2, f2);
    // flavour slots: -5..-1 -> 0..4, g -> 5, 1..5 -> 6..10; pairs u dbar, c sbar
    const float lf = fmaf(f1[7], f2[4], f1[9] * f2[2]);
    const float lb = fmaf(f1[4], f2[7], f1[2] * f2[9]);
    const float ishat = __builtin_amdgcn_rcpf(shat);
    return (double)(c.pref * (float)ltau * beta * ishat * pw * fmaf(kf, lf, kb * lb));
  }
};

}  // namespace vgx
