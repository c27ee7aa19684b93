// Internal helpers of libvgx: error reporting, Philox, wave reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdarg.h>
#include <string.h>

#include "../../include/vgx.h"

namespace vgx {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
vgx_status hip_fail(hipError_t e, const char* what, const char* file, int line);

#define VGX_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) return ::vgx::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

#define VGX_CHECK(cond, ...)                                                 \
  do {                                                                       \
    if (!(cond)) {                                                           \
      ::vgx::set_error(__VA_ARGS__);                                         \
      return VGX_EINVAL;                                                     \
    }                                                                        \
  } while (0)

#define VGX_TRY(expr)                                                        \
  do {                                                                       \
    vgx_status s_ = (expr);                                                  \
    if (s_ != VGX_OK) return s_;                                             \
  } while (0)

vgx_status dev_alloc(void** p, size_t bytes);
vgx_status host_alloc(void** p, size_t bytes);

// Number of compute units of the current device (cached per device).
int device_cus();

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon et al., SC'11).  Round on (c0,c1,c2,c3), key (k0,k1):
//   (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2,
//   c' = (hi1^c1^k0, lo1, hi0^c3^k1, lo0);  key += (W0, W1) between rounds.
// ---------------------------------------------------------------------------
struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    // three-input XOR in one v_bitop3_b32 (truth table 0x96)
    c0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
    c1 = lo1;
    c2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return {c0, c1, c2, c3};
}

// u = (k + 1/2) 2^-32, exact in FP64, strictly inside (0, 1).
__device__ __forceinline__ double word_to_unit(uint32_t k) {
  // k 2^-32 has at most 32 significant bits, so k 2^-32 + 2^-33 is exact:
  // one FMA gives (k + 1/2) 2^-32 bit for bit
  return fma((double)k, 0x1p-32, 0x1p-33);
}

// Uniforms of dims [0, D) of sample i; block b covers dims 4b..4b+3.
template <int D>
__device__ __forceinline__ void philox_uniforms(uint64_t i, uint32_t it, uint32_t stream_id, uint32_t k0,
                                                uint32_t k1, double (&u)[D]) {
#pragma unroll
  for (int b = 0; b < (D + 3) / 4; ++b) {
    const u32x4 w = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), it, (stream_id << 8) | (uint32_t)b, k0, k1);
    if (4 * b + 0 < D) u[4 * b + 0 < D ? 4 * b + 0 : 0] = word_to_unit(w.x);
    if (4 * b + 1 < D) u[4 * b + 1 < D ? 4 * b + 1 : 0] = word_to_unit(w.y);
    if (4 * b + 2 < D) u[4 * b + 2 < D ? 4 * b + 2 : 0] = word_to_unit(w.z);
    if (4 * b + 3 < D) u[4 * b + 3 < D ? 4 * b + 3 : 0] = word_to_unit(w.w);
  }
}

// ---------------------------------------------------------------------------
// Compensated (Neumaier) accumulation in FP64.
// ---------------------------------------------------------------------------
struct Comp {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double v) {
    const double t = s + v;
    c += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};

// Wave (64-lane) sum of a double using cross-lane shuffles; lane 0 holds it.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

}  // namespace vgx
