// Fused LO pp -> t tbar integrand (FP32 arithmetic, kinematics set up in
// FP64) with the log-bicubic PDF lookup served from LDS.
//
// Thesis: master formula sigma = sum_ab int dPhi_n L(x1, x2) |M|^2 (MadFlow
// chapter), factorisation sigma = sum_ij int dx1 dx2 f_i f_j sigma_ij (PDF
// chapter), sub-processes q qbar -> t tbar and g g -> t tbar (pp -> t tbar
// example), two-body phase space (phase-space section).  Matrix elements:
// the spin/colour-averaged LO forms (Combridge 1979; Ellis-Stirling-Webber
// Ch. 10) with tau_{1,2} = (1 -/+ beta cos)/2, rho = 4 m^2/s_hat:
//   |M|^2_qq = g^4 (4/9)(tau1^2 + tau2^2 + rho/2)
//   |M|^2_gg = g^4 (1/(6 tau1 tau2) - 3/8)(tau1^2 + tau2^2 + rho - rho^2/(4 tau1 tau2)).
// Map of the unit cube: tau = tau0^(1-x1), y = (x2 - 1/2) ln(1/tau),
// cos = 2 x3 - 1, so that
//   F = [J_tau/tau] J_y J_c * L * beta/(32 pi s_hat) * (hbar c)^2
//     = 2 L0 l_tau beta/(32 pi s tau) * (lum_gg |M|^2_gg + lum_qq |M|^2_qq) * conv,
// with L0 = ln(1/tau0), l_tau = ln(1/tau) = (1 - x1) L0 and the luminosities
// built from xf (f(x) = xf/x gives the 1/tau of dx1 dx2 = dtau dy).
//
// Rounding-safe forms (exact identities, no cancellation in FP32):
//   rho = exp(-x1 L0), beta^2 = -expm1(-x1 L0),
//   1 - beta cos = (1 - beta) + 2 beta (1 - x3),  1 + beta cos = (1 - beta) + 2 beta x3,
//   1 - beta = rho/(1 + beta),  ln x_{1,2} = +/- y - l_tau/2  (no log needed).
//
// PDF lookup: PdfRows (pdf_rows.h) at the fixed scale mu^2 = m_t^2.
#pragma once

#include "common.h"
#include "pdf_rows.h"

namespace vgx {

struct TTbarConst {
  // kinematics (FP64, set on the host from sqrt_s, m_t, alpha_s, conv)
  double L0;        // ln(1/tau0)
  float pref;       // 2 conv / (32 pi s)
  float g4;         // (4 pi alpha_s)^2
  PdfRowsConst pdf; // PDF rows at mu^2 = m_t^2, staged from x >= tau0
};

__host__ __device__ inline int ttbar_lds_floats(int nxs) { return pdf_rows_lds_floats(nxs); }

struct TTbar {
  static constexpr bool kStage = true;
  // five waves per SIMD (<= 96 VGPRs) measured faster than four
  static constexpr int kMinWaves = 5;
  TTbarConst c;
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
    // kinematics in FP64 (a handful of operations), then FP32
    const double v = x[0] * c.L0;                  // u1 L0
    const double ltau = (1.0 - x[0]) * c.L0;       // ln(1/tau)
    const double y = (x[1] - 0.5) * ltau;
    const float a1 = (float)(y - 0.5 * ltau);      // ln x1
    const float a2 = (float)(-y - 0.5 * ltau);     // ln x2
    const float w3 = (float)(1.0 - x[2]);          // 1 - u3
    const float u3 = (float)x[2];
    const float vf = (float)v;
    // v <= L0 (about 7.3 at 13 TeV): exp through the hardware exp2 loses at
    // most |v| 2^-24 relative, well inside the FP32 integrand's tolerance;
    // expm1 keeps full precision where beta -> 0.  Reciprocals use the
    // hardware rcp (1 ulp).
    const float rho = __expf(-vf);
    const float beta = __builtin_amdgcn_sqrtf(-expm1f(-vf));  // hardware sqrt, 1 ulp
    const float omb = rho * __builtin_amdgcn_rcpf(1.f + beta);  // 1 - beta
    const float tau1 = 0.5f * (omb + 2.f * beta * w3);
    const float tau2 = 0.5f * (omb + 2.f * beta * u3);
    const float t12 = tau1 * tau2;
    const float r12 = __builtin_amdgcn_rcpf(t12);
    const float ss = fmaf(tau1, tau1, tau2 * tau2);
    const float m_qq = c.g4 * (4.f / 9.f) * fmaf(0.5f, rho, ss);
    const float m_gg = c.g4 * fmaf(r12, 1.f / 6.f, -0.375f) * (ss + rho - 0.25f * rho * rho * r12);
    float f1[TT_NF], f2[TT_NF];
    P.pdf_at(a1, f1);
    P.pdf_at(a2, f2);
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
