// Fused LO pp -> photon/Z -> l+ l- (Drell-Yan) integrand: FP32 arithmetic,
// kinematics set up in FP64, the PDF lookup served from LDS (PdfRows at the
// fixed scale mu^2 = M_Z^2).
//
// Thesis: master formula sigma = sum_ab int dPhi_n L(x1, x2) |M|^2 (MadFlow
// chapter) and factorisation (PDF chapter).  Matrix element: q qbar -> l- l+
// through a photon and a Z (massless fermions), helicity amplitudes
// |A_ij|^2 = e^4 (1 +/- cos)^2 |F_ij|^2 (+ for equal quark and lepton
// helicities), F_ij = Q_q Q_l + g_i^q g_j^l chi, chi = s_hat / (s_W^2 c_W^2
// (s_hat - M_Z^2 + i M_Z Gamma_Z)), spin and colour average 1/12, cos the
// angle between the quark and the l-.  Summed over helicities:
//   (1 + cos)^2 S_same + (1 - cos)^2 S_opp,  S = a0 + a1 Re chi + a2 |chi|^2,
// coefficients per quark type set on the host.  A quark from the second beam
// sees the l- at pi - theta (cos -> -cos).
// Map of the unit cube: tau = tau_lo (tau_hi/tau_lo)^x1, y = (x2 - 1/2) ln(1/tau),
// cos = 2 x3 - 1, so J/tau = 2 Lr ln(1/tau), Lr = ln(tau_hi/tau_lo), and
//   F = 2 Lr ln(1/tau) conv e^4/(12 32 pi) / s_hat,  s_hat = m_lo^2 exp(x1 Lr),
//       * sum_q [xq(x1) xqbar(x2) A_q(cos) + xqbar(x1) xq(x2) A_q(-cos)].
// Rounding-safe forms: 1 + cos = 2 x3, 1 - cos = 2 (1 - x3).
#pragma once

#include "common.h"
#include "pdf_rows.h"

namespace vgx {

struct DYConst {
  double Llo;       // ln(1/tau_lo)
  double Lr;        // ln(tau_hi/tau_lo)
  double mlo2;      // m_lo^2 = tau_lo s
  double mz2d;      // M_Z^2
  float pref;       // 2 Lr conv e^4 / (12 32 pi)
  float mg2;        // (M_Z Gamma_Z)^2
  float kap;        // 1/(s_W^2 c_W^2)
  // helicity-sum coefficients [up, down]: same (LL + RR), opposite (LR + RL)
  float a0[2], as1[2], as2[2], ao1[2], ao2[2];
  PdfRowsConst pdf; // PDF rows at mu^2 = M_Z^2, staged from x >= tau_lo
};

struct DrellYan {
  static constexpr bool kStage = true;
  DYConst c;
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
    const double ltau = c.Llo - x[0] * c.Lr;     // ln(1/tau)
    const double y = (x[1] - 0.5) * ltau;
    const float a1 = (float)(y - 0.5 * ltau);    // ln x1
    const float a2 = (float)(-y - 0.5 * ltau);   // ln x2
    const float lt = (float)ltau;
    // s_hat = m_lo^2 exp(x1 Lr) in FP64: near the pole the Breit-Wigner
    // multiplies the relative error of s_hat by up to M_Z/Gamma_Z (~36), so
    // s_hat - M_Z^2 is formed before rounding to FP32
    const double sh = c.mlo2 * exp(x[0] * c.Lr);
    const float dm = (float)(sh - c.mz2d);
    const float shat = (float)sh;
    const float ishat = __builtin_amdgcn_rcpf(shat);
    const float den = fmaf(dm, dm, c.mg2);
    const float k1 = c.kap * shat * __builtin_amdgcn_rcpf(den);
    const float rex = k1 * dm;                   // Re chi
    const float ax2 = k1 * (c.kap * shat);       // |chi|^2
    const float cp = 2.f * (float)x[2];          // 1 + cos
    const float cm = 2.f * (float)(1.0 - x[2]);  // 1 - cos
    const float cp2 = cp * cp, cm2 = cm * cm;
    float Af[2], Ab[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const float ss = fmaf(c.as2[k], ax2, fmaf(c.as1[k], rex, c.a0[k]));
      const float so = fmaf(c.ao2[k], ax2, fmaf(c.ao1[k], rex, c.a0[k]));
      Af[k] = fmaf(cp2, ss, cm2 * so);
      Ab[k] = fmaf(cm2, ss, cp2 * so);
    }
    float f1[TT_NF], f2[TT_NF];
    P.pdf_at(a1, f1);
    P.pdf_at(a2, f2);
    // flavour slots: -5..-1 -> 0..4, g -> 5, 1..5 -> 6..10
    const float up_f = fmaf(f1[7], f2[3], f1[9] * f2[1]);     // u ubar + c cbar (quark from beam 1)
    const float up_b = fmaf(f1[3], f2[7], f1[1] * f2[9]);     // ubar u + cbar c
    const float dn_f = fmaf(f1[6], f2[4], fmaf(f1[8], f2[2], f1[10] * f2[0]));
    const float dn_b = fmaf(f1[4], f2[6], fmaf(f1[2], f2[8], f1[0] * f2[10]));
    const float sum = fmaf(Af[0], up_f, fmaf(Ab[0], up_b, fmaf(Af[1], dn_f, Ab[1] * dn_b)));
    return (double)(c.pref * lt * ishat * sum);
  }
};

}  // namespace vgx
