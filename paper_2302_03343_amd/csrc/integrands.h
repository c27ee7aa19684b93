// Device integrands of libvgx.  Each integrand is a small struct with
//   static constexpr int lds_doubles(...)  -- extra LDS it stages (in doubles)
//   __device__ void stage(double* lds)      -- cooperative LDS staging
//   __device__ double eval(const double (&x)[D]) const
// Parameters live in a fixed-size by-value kernel argument.
#pragma once

#include "common.h"

namespace vgx {

constexpr int MAX_PARAMS = 2 * VGX_MAX_DIM + 4;

struct IntegrandParams {
  double p[MAX_PARAMS];
};

// Integrands without LDS staging share this no-op.
struct NoStage {
  static constexpr bool kStage = false;
  __device__ __forceinline__ void stage(float*) {}
};

// prod_j N(x_j; c_j, s_j), each factor normalised on R.  One exp of the
// summed exponent; the normalisation prod 1/(s_j sqrt(2 pi)) is folded on
// the host into p[2D] so that the device does only the data-dependent part.
template <int D, typename R>
struct Gauss : NoStage {
  IntegrandParams prm;  // [c_0..c_{D-1}, 1/(s_j sqrt 2) .., norm]
  __device__ __forceinline__ double eval(const double (&x)[D]) const {
    R e = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      // z = (x - c) k as x k - c k (one FMA; c k is loop-invariant)
      const R k = (R)prm.p[D + j];
      const R z = fma((R)x[j], k, -((R)prm.p[j] * k));
      e = fma(z, z, e);
    }
    return (double)((R)prm.p[2 * D] * exp(-e));
  }
};

// Genz oscillatory: cos(2 pi w_1 + sum_j c_j x_j).  p = [2 pi w_1, c_0 ..].
template <int D, typename R>
struct GenzOsc : NoStage {
  IntegrandParams prm;
  __device__ __forceinline__ double eval(const double (&x)[D]) const {
    R a = (R)prm.p[0];
#pragma unroll
    for (int j = 0; j < D; ++j) a = fma((R)prm.p[1 + j], (R)x[j], a);
    return (double)cos(a);
  }
};

// Genz product peak: prod_j (c_j^-2 + (x_j - w_j)^2)^-1.
// p = [w_0..w_{D-1}, c_0^-2 .. c_{D-1}^-2].
template <int D, typename R>
struct GenzPeak : NoStage {
  IntegrandParams prm;
  __device__ __forceinline__ double eval(const double (&x)[D]) const {
    R den = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const R z = (R)x[j] - (R)prm.p[j];
      den *= fma(z, z, (R)prm.p[D + j]);
    }
    return (double)((R)1 / den);
  }
};

}  // namespace vgx
