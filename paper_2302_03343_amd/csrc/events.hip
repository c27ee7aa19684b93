// Event generation: RAMBO phase-space points and acceptance-rejection
// unweighting.
//
// Thesis: MC chapter (RAMBO subsection, acceptance-rejection paragraph) and
// the MadFlow chapter (vectorised RAMBO phase-space generator; unweighted
// event exporter: keep an event when its weight exceeds a uniform number times
// the sample's largest weight).
//
// RAMBO: one event per thread, the n momenta in registers (n is a template
// parameter, 2..VGX_MAX_PART); outputs structure-of-arrays [4][n][N] so that
// every store of a wave is contiguous.  Uniforms: Philox-4x32-10 with the
// counter of sample e of the VEGAS kernels (low and high words of e, the
// iteration, stream << 8 | block), block i giving particle i's four numbers.
// Massive momenta: xi by Newton's method from xi0 = sqrt(1 - (sum m/sqrt s)^2),
// where the (convex, increasing) constraint is >= 0, so the iterates approach
// the root from above.  The constraint is evaluated in FP64; its derivative
// only sets the step length and takes the hardware reciprocal (relative error
// about 2^-23), which keeps the convergence quadratic down to 2^-23 of the
// step.  The loop ends after a step below 2^-30 of xi: the error left is then
// of the order of xi's own rounding.
//
// Unweighting: w_max by a max over the positive weights (block maxima, then
// one workgroup over those: exact in any order);
// then kept indices in ascending order by a three-pass compaction: per-block
// counts (keeping each wave's ballot of its decisions), one exclusive scan,
// and a scatter that ranks the kept events from the ballots.
#include "common.h"

#include <math.h>
#include <string.h>

#include <mutex>

namespace vgx {

constexpr int RB_BLOCK = 256;

struct RamboArgs {
  int64_t n_events, first;
  double sqrt_s, w0, w0m, sum_m;  // w0m = w0 s^(2-n), the massive weight's constant
  double m[VGX_MAX_PART];
  uint32_t k0, k1, sid, it;
};

// x^k for a compile-time k >= 0, by repeated squaring
template <int K>
__device__ __forceinline__ double ipow(double x) {
  if constexpr (K == 0)
    return 1.0;
  else if constexpr (K == 1)
    return x;
  else {
    const double h = ipow<K / 2>(x * x);
    if constexpr (K % 2) return h * x;
    return h;
  }
}

template <int N, bool MASSIVE>
__global__ __launch_bounds__(RB_BLOCK) void k_rambo(RamboArgs a, double* __restrict__ mom, double* __restrict__ wout) {
  const int64_t stride = (int64_t)gridDim.x * RB_BLOCK;
  for (int64_t e = (int64_t)blockIdx.x * RB_BLOCK + threadIdx.x; e < a.n_events; e += stride) {
    const uint64_t idx = (uint64_t)(a.first + e);
    double q[N][4];
    double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0, Q3 = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const u32x4 r = philox4x32_10((uint32_t)idx, (uint32_t)(idx >> 32), a.it, (a.sid << 8) | (uint32_t)i, a.k0, a.k1);
      const double c = 2.0 * word_to_unit(r.x) - 1.0;
      const double e0 = -log(word_to_unit(r.z) * word_to_unit(r.w));
      const double st = sqrt(1.0 - c * c);
      double sn, cs;
      sincospi(2.0 * word_to_unit(r.y), &sn, &cs);  // phi = 2 pi u, without a reduction modulo 2 pi
      q[i][0] = e0;
      q[i][1] = e0 * st * cs;
      q[i][2] = e0 * st * sn;
      q[i][3] = e0 * c;
      Q0 += q[i][0];
      Q1 += q[i][1];
      Q2 += q[i][2];
      Q3 += q[i][3];
    }
    // boost and scale onto P = (sqrt s, 0): p = x H_b(q)
    const double M = sqrt(Q0 * Q0 - Q1 * Q1 - Q2 * Q2 - Q3 * Q3);
    const double iM = 1.0 / M;
    const double b1 = -Q1 * iM, b2 = -Q2 * iM, b3 = -Q3 * iM;
    const double x = a.sqrt_s * iM, gam = Q0 * iM, aa = 1.0 / (1.0 + gam);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double bq = b1 * q[i][1] + b2 * q[i][2] + b3 * q[i][3];
      const double q0 = q[i][0];
      q[i][0] = x * (gam * q0 + bq);
      q[i][1] = x * (q[i][1] + b1 * q0 + aa * bq * b1);
      q[i][2] = x * (q[i][2] + b2 * q0 + aa * bq * b2);
      q[i][3] = x * (q[i][3] + b3 * q0 + aa * bq * b3);
    }
    double w = a.w0;
    if constexpr (MASSIVE) {
      // sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt s
      const double t = a.sum_m / a.sqrt_s;
      double xi = sqrt(1.0 - t * t);
      for (int iter = 0; iter < 64; ++iter) {
        double f = -a.sqrt_s, fp = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const double xe = xi * q[i][0];
          const double k0 = sqrt(a.m[i] * a.m[i] + xe * xe);
          f += k0;
          fp += xe * q[i][0] * __builtin_amdgcn_rcp(k0);
        }
        const double step = f * __builtin_amdgcn_rcp(fp);
        xi -= step;
        if (!(fabs(step) >= 0x1p-30 * xi)) break;
      }
      double sk = 0.0, pr = 1.0, sk2 = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double kabs = xi * q[i][0];  // |k_i| = xi |p_i| = xi p_i^0 (p_i massless)
        const double k0 = sqrt(a.m[i] * a.m[i] + kabs * kabs);
        const double ik = 1.0 / k0;
        sk += kabs;
        pr *= kabs * ik;
        sk2 += kabs * kabs * ik;
        q[i][0] = k0;
        q[i][1] *= xi;
        q[i][2] *= xi;
        q[i][3] *= xi;
      }
      w = a.w0m * (ipow<2 * N - 3>(sk) * pr / sk2);
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) mom[((int64_t)c * N + i) * a.n_events + e] = q[i][c];
    wout[e] = w;
  }
}

// ---------------------------------------------------------------------------
// Unweighting
// ---------------------------------------------------------------------------
constexpr int UW_BLOCK = 256;
constexpr int UW_ROUNDS = 16;
constexpr int UW_CHUNK = UW_BLOCK * UW_ROUNDS;  // events per block, ranked in order

// Largest weight: a block maximum per workgroup into part[], then one
// workgroup reduces part[] (one atomic per workgroup on a single address
// serialised at the memory: about 30 us for 2048 workgroups).
__global__ __launch_bounds__(UW_BLOCK) void k_uw_max(int64_t n, const double* __restrict__ w,
                                                     double* __restrict__ part) {
  __shared__ double red[UW_BLOCK / 64];
  double m = 0.0;
  // 16-byte loads, four in flight per lane (one 8-byte load per lane and
  // round left the kernel waiting on HBM latency); a weight before the first
  // 16-byte boundary and an odd one at the end are read by thread 0
  const int64_t head = ((uintptr_t)w & 15) ? 1 : 0;
  const int64_t n2 = n > head ? (n - head) >> 1 : 0;
  const double2* w2 = (const double2*)(w + head);
  const int64_t stride = (int64_t)gridDim.x * UW_BLOCK;
  int64_t i = (int64_t)blockIdx.x * UW_BLOCK + threadIdx.x;
  for (; i + 3 * stride < n2; i += 4 * stride) {
    double2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = w2[i + k * stride];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      m = v[k].x > m ? v[k].x : m;  // NaN and non-positive weights never win
      m = v[k].y > m ? v[k].y : m;
    }
  }
  for (; i < n2; i += stride) {
    const double2 v = w2[i];
    m = v.x > m ? v.x : m;
    m = v.y > m ? v.y : m;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double h = head ? w[0] : 0.0;
    const double t = head + 2 * n2 < n ? w[n - 1] : 0.0;
    m = h > m ? h : m;
    m = t > m ? t : m;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < UW_BLOCK / 64; ++k) m = red[k] > m ? red[k] : m;
    part[blockIdx.x] = m;
  }
}

constexpr int UW_FINAL = 1024;

__global__ __launch_bounds__(UW_FINAL) void k_uw_max_final(int nparts, const double* __restrict__ part,
                                                           unsigned long long* __restrict__ out_bits) {
  __shared__ double red[UW_FINAL / 64];
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += UW_FINAL) m = part[i] > m ? part[i] : m;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < UW_FINAL / 64; ++k) m = red[k] > m ? red[k] : m;
    *out_bits = (unsigned long long)__double_as_longlong(m);  // m >= 0: its bit pattern orders like it
  }
}

struct UwArgs {
  int64_t n;
  double w_max;  // > 0: given; else read from w_max_bits
  uint32_t k0, k1, sid, it;
};

// The accept number of event i: word 0 of Philox block 0xFF of sample i.  The
// samplers use blocks 0 .. (4-word blocks they need) - 1 (at most 10 here), so
// an accept number never coincides with a number that made the event.
constexpr uint32_t UW_PHILOX_BLOCK = 0xFFu;

__device__ __forceinline__ bool uw_keep(const UwArgs& a, const double* w, int64_t i, double wmax) {
  const u32x4 r = philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), a.it, (a.sid << 8) | UW_PHILOX_BLOCK,
                                a.k0, a.k1);
  return w[i] > word_to_unit(r.x) * wmax;
}

__device__ __forceinline__ double uw_wmax(const UwArgs& a, const unsigned long long* bits) {
  return a.w_max > 0.0 ? a.w_max : __longlong_as_double((long long)*bits);
}

// The keep decisions of a block as UW_MASKS wave ballots, in event order
// (mask r * 4 + wave covers events base + 256 r + 64 wave + lane), for the
// scatter; and the block's count.
constexpr int UW_MASKS = UW_ROUNDS * (UW_BLOCK / 64);
static_assert(UW_MASKS == 64, "the scatter scans a block's masks within one wave");

__global__ __launch_bounds__(UW_BLOCK) void k_uw_count(UwArgs a, const double* __restrict__ w,
                                                       const unsigned long long* __restrict__ bits,
                                                       int64_t* __restrict__ counts,
                                                       unsigned long long* __restrict__ masks) {
  __shared__ int red[UW_BLOCK / 64];
  const double wmax = uw_wmax(a, bits);
  const int64_t base = (int64_t)blockIdx.x * UW_CHUNK;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int c = 0;
  for (int r = 0; r < UW_ROUNDS; ++r) {
    const int64_t i = base + r * UW_BLOCK + threadIdx.x;
    const bool keep = i < a.n && uw_keep(a, w, i, wmax);
    const unsigned long long m = __ballot(keep);
    if (lane == 0) masks[(int64_t)blockIdx.x * UW_MASKS + r * (UW_BLOCK / 64) + wv] = m;
    c += keep ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < UW_BLOCK / 64; ++k) t += red[k];
    counts[blockIdx.x] = t;
  }
}

// Exclusive scan of the block counts in place (one workgroup of 1024), the
// total in counts[nb].
__global__ __launch_bounds__(1024) void k_uw_scan(int64_t nb, int64_t* __restrict__ counts,
                                                 int64_t* __restrict__ total_out) {
  __shared__ int64_t part[1024 / 64];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? counts[i] : 0;
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    int64_t before = carry;
    for (int k = 0; k < wv; ++k) before += part[k];
    if (i < nb) counts[i] = before + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[nb] = carry;
    *total_out = carry;  // beside the max's bits: one read-back for both
  }
}

// Kept indices from the block's masks: lane j of every wave holds mask j and
// the exclusive prefix of the popcounts, so the position of each kept event
// needs no workgroup barrier; the weights are not read again.
__global__ __launch_bounds__(UW_BLOCK) void k_uw_scatter(int64_t n, const unsigned long long* __restrict__ masks,
                                                         const int64_t* __restrict__ offsets,
                                                         int64_t* __restrict__ idx_out) {
  const int64_t base = (int64_t)blockIdx.x * UW_CHUNK;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long mj = masks[(int64_t)blockIdx.x * UW_MASKS + lane];
  const int cj = __popcll(mj);
  int incl = cj;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  const int excl = incl - cj;
  const uint32_t mlo = (uint32_t)mj, mhi = (uint32_t)(mj >> 32);
  const int64_t pos = offsets[blockIdx.x];
  for (int r = 0; r < UW_ROUNDS; ++r) {
    const int j = r * (UW_BLOCK / 64) + wv;
    const uint32_t lo = (uint32_t)__shfl((int)mlo, j, 64), hi = (uint32_t)__shfl((int)mhi, j, 64);
    const int pre = __shfl(excl, j, 64);
    const bool keep = lane < 32 ? (lo >> lane) & 1u : (hi >> (lane - 32)) & 1u;
    const int rank = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
    const int64_t i = base + r * UW_BLOCK + threadIdx.x;
    if (keep && i < n) idx_out[pos + pre + rank] = i;
  }
}

template <int N>
void launch_rambo(const RamboArgs& a, bool massive, int grid, hipStream_t st, double* mom, double* w) {
  if (massive)
    hipLaunchKernelGGL((k_rambo<N, true>), dim3(grid), dim3(RB_BLOCK), 0, st, a, mom, w);
  else
    hipLaunchKernelGGL((k_rambo<N, false>), dim3(grid), dim3(RB_BLOCK), 0, st, a, mom, w);
}

}  // namespace vgx

using namespace vgx;

extern "C" vgx_status rambo_generate(int32_t n_part, const double* masses, double sqrt_s, uint64_t seed,
                                     uint32_t stream_id, uint32_t iteration, int64_t first, int64_t n_events,
                                     double* mom_dev, double* w_dev, void* stream) {
  VGX_CHECK(n_part >= 2 && n_part <= VGX_MAX_PART, "rambo_generate: n_part %d out of 2..%d", n_part, VGX_MAX_PART);
  VGX_CHECK(masses, "rambo_generate: null masses");
  VGX_CHECK(sqrt_s > 0.0 && isfinite(sqrt_s), "rambo_generate: sqrt_s must be positive and finite");
  VGX_CHECK(stream_id < (1u << 24), "rambo_generate: stream_id must be < 2^24");
  VGX_CHECK(first >= 0 && n_events >= 0, "rambo_generate: negative first or n_events");
  RamboArgs a{};
  a.n_events = n_events;
  a.first = first;
  a.sqrt_s = sqrt_s;
  bool massive = false;
  for (int i = 0; i < n_part; ++i) {
    VGX_CHECK(masses[i] >= 0.0 && isfinite(masses[i]), "rambo_generate: mass %d must be >= 0 and finite", i);
    a.m[i] = masses[i];
    a.sum_m += masses[i];
    massive = massive || masses[i] > 0.0;
  }
  VGX_CHECK(a.sum_m < sqrt_s, "rambo_generate: the masses (sum %g) do not fit in sqrt_s = %g", a.sum_m, sqrt_s);
  if (n_events == 0) return VGX_OK;
  VGX_CHECK(mom_dev && w_dev, "rambo_generate: null device pointer");
  const int n = n_part;
  const double s = sqrt_s * sqrt_s;
  // w0 = (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / (Gamma(n) Gamma(n-1))
  a.w0m = pow(2.0 * M_PI, 4.0 - 3.0 * n) * pow(M_PI / 2.0, n - 1.0) / (tgamma((double)n) * tgamma(n - 1.0));
  a.w0 = a.w0m * pow(s, n - 2.0);
  a.k0 = (uint32_t)seed;
  a.k1 = (uint32_t)(seed >> 32);
  a.sid = stream_id;
  a.it = iteration;
  const int64_t want = (n_events + RB_BLOCK - 1) / RB_BLOCK;
  const int grid = (int)(want < (int64_t)device_cus() * 16 ? want : (int64_t)device_cus() * 16);
  hipStream_t st = (hipStream_t)stream;
  switch (n_part) {
    case 2: launch_rambo<2>(a, massive, grid, st, mom_dev, w_dev); break;
    case 3: launch_rambo<3>(a, massive, grid, st, mom_dev, w_dev); break;
    case 4: launch_rambo<4>(a, massive, grid, st, mom_dev, w_dev); break;
    case 5: launch_rambo<5>(a, massive, grid, st, mom_dev, w_dev); break;
    case 6: launch_rambo<6>(a, massive, grid, st, mom_dev, w_dev); break;
    case 7: launch_rambo<7>(a, massive, grid, st, mom_dev, w_dev); break;
    case 8: launch_rambo<8>(a, massive, grid, st, mom_dev, w_dev); break;
    case 9: launch_rambo<9>(a, massive, grid, st, mom_dev, w_dev); break;
    default: launch_rambo<10>(a, massive, grid, st, mom_dev, w_dev); break;
  }
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

namespace {

// Scratch of one unweighting call: the max's bit pattern and the kept count,
// nb + 1 block counts (scanned in place), the max search's block maxima,
// nb x UW_MASKS keep masks (one bit per event).  Every word is written
// before it is read, so nothing needs clearing; the bits are written by
// k_uw_max_final when the maximum is searched and not read otherwise.
size_t uw_scratch_bytes(int64_t nb, int grid) {
  return sizeof(unsigned long long) * (2 + (size_t)nb * UW_MASKS) + sizeof(int64_t) * (size_t)(nb + 1) +
         sizeof(double) * (size_t)grid;
}

struct UwPlan {
  int64_t nb;
  int grid;
};

vgx_status uw_check(int64_t n, const double* w_dev, double w_max, uint32_t stream_id, int64_t* idx_dev,
                    int64_t* n_kept, double* w_max_used, const char* who, UwPlan* plan, bool* done) {
  VGX_CHECK(n >= 0, "%s: n < 0", who);
  VGX_CHECK(n_kept, "%s: null n_kept", who);
  VGX_CHECK(stream_id < (1u << 24), "%s: stream_id must be < 2^24", who);
  VGX_CHECK(!(w_max < 0.0) && !isnan(w_max), "%s: w_max must be >= 0 (0: the sample's maximum)", who);
  *n_kept = 0;
  *done = false;
  if (n == 0) {
    if (w_max_used) *w_max_used = w_max;
    *done = true;
    return VGX_OK;
  }
  VGX_CHECK(w_dev && idx_dev, "%s: null device pointer", who);
  plan->nb = (n + UW_CHUNK - 1) / UW_CHUNK;
  VGX_CHECK(plan->nb < (int64_t)1 << 31, "%s: n too large", who);
  const int64_t want = (n + UW_BLOCK - 1) / UW_BLOCK;
  plan->grid = (int)(want < (int64_t)device_cus() * 8 ? want : (int64_t)device_cus() * 8);
  return VGX_OK;
}

// Enqueue the unweighting kernels on buf (uw_scratch_bytes) and the
// read-back of the max's bits and the kept count into hb.
hipError_t uw_enqueue(const UwPlan& p, int64_t n, const double* w_dev, double w_max, uint64_t seed,
                      uint32_t stream_id, uint32_t iteration, int64_t* idx_dev, void* buf, hipStream_t st,
                      unsigned long long (&hb)[2]) {
  unsigned long long* bits = (unsigned long long*)buf;
  int64_t* total_dev = (int64_t*)(bits + 1);
  int64_t* counts = total_dev + 1;
  double* part = (double*)(counts + p.nb + 1);
  unsigned long long* masks = (unsigned long long*)(part + p.grid);
  UwArgs a{n, w_max, (uint32_t)seed, (uint32_t)(seed >> 32), stream_id, iteration};
  if (!(w_max > 0.0)) {
    hipLaunchKernelGGL(k_uw_max, dim3(p.grid), dim3(UW_BLOCK), 0, st, n, w_dev, part);
    hipLaunchKernelGGL(k_uw_max_final, dim3(1), dim3(UW_FINAL), 0, st, p.grid, part, bits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_uw_count, dim3((unsigned)p.nb), dim3(UW_BLOCK), 0, st, a, w_dev, bits, counts, masks);
  hipLaunchKernelGGL(k_uw_scan, dim3(1), dim3(1024), 0, st, p.nb, counts, total_dev);
  hipLaunchKernelGGL(k_uw_scatter, dim3((unsigned)p.nb), dim3(UW_BLOCK), 0, st, n, masks, counts, idx_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(hb, bits, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
}

void uw_results(const unsigned long long (&hb)[2], double w_max, int64_t* n_kept, double* w_max_used) {
  *n_kept = (int64_t)hb[1];
  if (w_max_used) {
    double wm;
    memcpy(&wm, &hb[0], sizeof(wm));
    *w_max_used = w_max > 0.0 ? w_max : wm;
  }
}

}  // namespace

extern "C" vgx_status unweight(int64_t n, const double* w_dev, double w_max, uint64_t seed, uint32_t stream_id,
                               uint32_t iteration, int64_t* idx_dev, int64_t* n_kept, double* w_max_used,
                               void* stream) {
  UwPlan p{};
  bool done = false;
  VGX_TRY(uw_check(n, w_dev, w_max, stream_id, idx_dev, n_kept, w_max_used, "unweight", &p, &done));
  if (done) return VGX_OK;
  hipStream_t st = (hipStream_t)stream;
  void* buf = nullptr;  // stream-ordered
  VGX_HIP(hipMallocAsync(&buf, uw_scratch_bytes(p.nb, p.grid), st));
  unsigned long long hb[2] = {0, 0};  // the max's bits, the kept count
  hipError_t e = uw_enqueue(p, n, w_dev, w_max, seed, stream_id, iteration, idx_dev, buf, st, hb);
  hipError_t ef = hipFreeAsync(buf, st);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "unweight", __FILE__, __LINE__);
  uw_results(hb, w_max, n_kept, w_max_used);
  return VGX_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free unweighting: the same kernels on a fixed device array.
// ---------------------------------------------------------------------------
// One copy per GPU, held until the process ends.  In host code the name is
// a host-side stand-in, not a device address: host code uses only the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[VGX_UNWEIGHT_STATIC_BYTES];

namespace {

constexpr int UW_MAX_DEVICES = 64;
std::mutex g_uw_mu;
void* g_uw_scratch[UW_MAX_DEVICES] = {};

// The current device's address of the array, looked up once per device.
vgx_status uw_static_scratch(void** out) {
  int dev = 0;
  VGX_HIP(hipGetDevice(&dev));
  VGX_CHECK(dev >= 0 && dev < UW_MAX_DEVICES, "unweight_noalloc: device %d beyond %d", dev, UW_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_uw_mu);
  if (!g_uw_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error("unweight_noalloc: hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
                hipGetErrorString(e));
      return VGX_EDEVICE;
    }
    g_uw_scratch[dev] = p;
  }
  *out = g_uw_scratch[dev];
  return VGX_OK;
}

}  // namespace

extern "C" vgx_status unweight_noalloc(int64_t n, const double* w_dev, double w_max, uint64_t seed,
                                       uint32_t stream_id, uint32_t iteration, int64_t* idx_dev, int64_t* n_kept,
                                       double* w_max_used, void* stream) {
  UwPlan p{};
  bool done = false;
  VGX_TRY(uw_check(n, w_dev, w_max, stream_id, idx_dev, n_kept, w_max_used, "unweight_noalloc", &p, &done));
  if (done) return VGX_OK;
  VGX_CHECK(n <= VGX_UNWEIGHT_NOALLOC_MAX && uw_scratch_bytes(p.nb, p.grid) <= VGX_UNWEIGHT_STATIC_BYTES,
            "unweight_noalloc: n = %lld needs %zu bytes of scratch, beyond the fixed %d (at most %lld events)",
            (long long)n, uw_scratch_bytes(p.nb, p.grid), VGX_UNWEIGHT_STATIC_BYTES,
            (long long)VGX_UNWEIGHT_NOALLOC_MAX);
  void* buf = nullptr;
  VGX_TRY(uw_static_scratch(&buf));
  hipStream_t st = (hipStream_t)stream;
  unsigned long long hb[2] = {0, 0};
  hipError_t e = uw_enqueue(p, n, w_dev, w_max, seed, stream_id, iteration, idx_dev, buf, st, hb);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "unweight_noalloc", __FILE__, __LINE__);
  uw_results(hb, w_max, n_kept, w_max_used);
  return VGX_OK;
}
