// Pieces of the VEGAS path shared by the single-integral kernels
// (vegas.hip) and the batched persistent kernel (batch.hip): the grid map,
// the per-iteration record and its inverse-variance combination, Lepage's
// refinement of one dimension, and the context structure.
#pragma once

#include "common.h"
#include "integrands.h"
#include "ttbar.h"
#include "drellyan.h"
#include "singletop.h"
#include "ttbar_dyn.h"

namespace vgx {

struct IterRecord {
  double mean, var, s1, s2;
  int64_t n;
  int32_t finite;
  int32_t pad;
};

struct Combined {
  double mean, sigma, chi2_dof;
  int32_t n_used;
  int32_t pad;
};

constexpr int MAX_RECORDS = 4096;

// Grid map (inverse transform through the piecewise-constant density of the
// bins): i = min(floor(u N), N-1), delta = u N - i,
// x = e_i + delta (e_{i+1} - e_i), J = prod_j N (e_{i+1} - e_i).
template <int D>
__device__ __forceinline__ double grid_map(const double (&u)[D], const double* se, int nb, double (&x)[D],
                                           int (&idx)[D]) {
  double jac = 1.0;
  const double dnb = (double)nb;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const double t = u[j] * dnb;
    int i = (int)t;
    i = i < nb - 1 ? i : nb - 1;
    i = i > 0 ? i : 0;  // points given by the caller may sit on or outside the cube's faces
    const double delta = t - (double)i;
    const double lo = se[j * (nb + 1) + i];
    const double w = se[j * (nb + 1) + i + 1] - lo;
    x[j] = fma(delta, w, lo);
    jac *= dnb * w;
    idx[j] = i;
  }
  return jac;
}

// The same map with the edge pairs of the odd dimensions read from global
// memory (one 16-byte load, served by the L1: the grid is a few KB) instead
// of LDS, for kernels whose LDS is their limit and whose vector-memory path
// is otherwise idle.  The edges are the same, so is the result.
typedef double double2_a8 __attribute__((ext_vector_type(2), aligned(8)));
template <int D>
__device__ __forceinline__ double grid_map_split(const double (&u)[D], const double* se,
                                                 const double* __restrict__ ge, int nb, double (&x)[D],
                                                 int (&idx)[D]) {
  double jac = 1.0;
  const double dnb = (double)nb;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const double t = u[j] * dnb;
    int i = (int)t;
    i = i < nb - 1 ? i : nb - 1;
    i = i > 0 ? i : 0;
    const double delta = t - (double)i;
    double lo, w;
    if (j & 1) {
      const double2_a8 e = *(const double2_a8*)(ge + j * (nb + 1) + i);
      lo = e.x;
      w = e.y - lo;
    } else {
      lo = se[j * (nb + 1) + i];
      w = se[j * (nb + 1) + i + 1] - lo;
    }
    x[j] = fma(delta, w, lo);
    jac *= dnb * w;
    idx[j] = i;
  }
  return jac;
}

// The grid map from scaled coordinates t_j = u_j N (exactly representable
// for the sources here): i = floor(t), delta = t - i, x = e_i + delta w_i
// (w_i = e_{i+1} - e_i), J = N^D prod_j w_i with the factor N^D given as nbD.
// INTERIOR: the source guarantees 0 < t < N (Philox uniforms), so i needs no
// clamp and delta is fract(t); else i is clamped into [0, N-1] (caller
// points on or outside the cube's faces) and delta = t - i.  GLOBAL: the
// edge pairs come from global memory (one 16-byte load each, served by the
// L1: the grid is a few KB), else from LDS.  Integrands without LDS tables
// take GLOBAL: their LDS holds the histogram copies, whose atomics are the
// LDS's load; with the edges too it was the limit (d = 4 Gaussian, 1e9
// samples: 4.76 ms all in LDS, 4.00 ms with the odd dimensions in global
// memory, 3.83 ms with all of them).
template <int D, bool INTERIOR, bool GLOBAL>
__device__ __forceinline__ double grid_map_t(const double (&t)[D], const double* se, const double* __restrict__ ge,
                                             int nb, double nbD, double (&x)[D], int (&idx)[D]) {
  double jw = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    int i = (int)t[j];
    double delta;
    if constexpr (INTERIOR) {
      delta = __builtin_amdgcn_fract(t[j]);
    } else {
      i = i < nb - 1 ? i : nb - 1;
      i = i > 0 ? i : 0;
      delta = t[j] - (double)i;
    }
    double lo, w;
    if constexpr (GLOBAL) {
      // a 32-bit byte offset from the uniform base (a scalar-base load)
      const uint32_t off = (uint32_t)(j * (nb + 1) + i) * 8u;
      const double2_a8 e = *(const double2_a8*)((const char*)ge + off);
      lo = e.x;
      w = e.y - lo;
    } else {
      lo = se[j * (nb + 1) + i];
      w = se[j * (nb + 1) + i + 1] - lo;
    }
    x[j] = fma(delta, w, lo);
    jw *= w;
    idx[j] = i;
  }
  return jw * nbD;
}

// Butterfly merge of compensated sums over the 64 lanes of a wave, in a fixed
// order (partner distance 1, 2, 4, ..., 32).
__device__ __forceinline__ Comp wave_merge(Comp a) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const double os = __shfl_xor(a.s, m, 64), oc = __shfl_xor(a.c, m, 64);
    a.add(os);
    a.c += oc;
  }
  return a;
}

// Estimate of one iteration from its compensated sums, stored as record
// k_rec, then the inverse-variance combination of the finite records
// 0..k_rec with chi^2/dof:  E = S1/n, var(E) = max(S2/n - E^2, 0)/(n-1);
// E_bar = S^2 sum E_i/S_i^2, 1/S^2 = sum 1/S_i^2,
// chi^2/dof = sum (E_i - E_bar)^2/S_i^2/(M-1).  A zero variance makes that
// estimate exact (sigma 0).  Called by the 64 lanes of one wave, which split
// the records (lane l takes l, l+64, ...) so that the cost per iteration does
// not grow with the number of stored estimates; lane 0 writes the results.
__device__ inline void finalize_record(double s1, double s2, int64_t n, IterRecord* rec, int k_rec, Combined* comb) {
  // no contraction into FMAs, so that every kernel that inlines this gives the same bits
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  // this lane's first stored record (k = lane), read before record k_rec is
  // written so that the read overlaps the caller's
  double mean0 = 0.0, var0 = 0.0;
  bool fin0 = false;
  if (lane < k_rec) {
    mean0 = rec[lane].mean;
    var0 = rec[lane].var;
    fin0 = rec[lane].finite;
  }
  IterRecord r;
  r.s1 = s1;
  r.s2 = s2;
  r.n = n;
  r.mean = s1 / (double)n;
  const double m2 = s2 / (double)n - r.mean * r.mean;
  r.var = n > 1 ? (m2 > 0.0 ? m2 : 0.0) / (double)(n - 1) : 0.0;
  r.finite = isfinite(r.mean) && isfinite(r.var);
  r.pad = 0;
  if (lane == 0) rec[k_rec] = r;
  // record k_rec is taken from registers: the other lanes must not read
  // the store lane 0 has just issued
  auto mean_var = [&](int k, double& mean, double& var) -> bool {
    if (k == k_rec) { mean = r.mean; var = r.var; return r.finite; }
    if (k == lane) { mean = mean0; var = var0; return fin0; }
    mean = rec[k].mean;
    var = rec[k].var;
    return rec[k].finite;
  };
  int used = 0, zero_var = MAX_RECORDS;
  Comp wsum, msum;
  for (int k = lane; k <= k_rec; k += 64) {
    double mean, var;
    if (!mean_var(k, mean, var)) continue;
    ++used;
    if (var == 0.0) {
      zero_var = k < zero_var ? k : zero_var;
    } else {
      wsum.add(1.0 / var);
      msum.add(mean / var);
    }
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    used += __shfl_xor(used, m, 64);
    const int o = __shfl_xor(zero_var, m, 64);
    zero_var = o < zero_var ? o : zero_var;
  }
  Combined c{0.0, 0.0, 0.0, used, 0};
  if (zero_var < MAX_RECORDS) {
    double mean, var;
    mean_var(zero_var, mean, var);
    c.mean = mean;
  } else if (used > 0) {
    wsum = wave_merge(wsum);
    msum = wave_merge(msum);
    // lane 0's combination is the one written; every lane uses it
    c.mean = __shfl(msum.value() / wsum.value(), 0, 64);
    c.sigma = sqrt(1.0 / __shfl(wsum.value(), 0, 64));
    if (used > 1) {
      Comp chi;
      for (int k = lane; k <= k_rec; k += 64) {
        double mean, var;
        if (!mean_var(k, mean, var)) continue;
        const double dd = mean - c.mean;
        chi.add(dd * dd / var);
      }
      chi = wave_merge(chi);
      c.chi2_dof = chi.value() / (double)(used - 1);
    }
  }
  if (lane == 0) *comb = c;
}

// Lepage's refinement of one dimension, by one 64-thread workgroup:
// 3-point smoothing of the accumulated (f J)^2 per bin, normalisation to
// p_i, damping r_i = ((1 - p_i)/ln(1/p_i))^alpha, re-binning to equal shares
// of sum r with r spread uniformly inside each old bin.  A dimension whose
// histogram is all zero, or not finite (an iteration with a non-finite
// weight, which the combination excludes too), is left unchanged.
__device__ inline void refine_dim(double* __restrict__ ej, const double* __restrict__ hj, int nb, double alpha) {
  __shared__ double d[VGX_MAX_BINS], r[VGX_MAX_BINS], cum[VGX_MAX_BINS + 1], e[VGX_MAX_BINS + 1];
  __shared__ double tot_d, tot_sm;
  for (int i = threadIdx.x; i < nb; i += 64) d[i] = hj[i];
  for (int i = threadIdx.x; i <= nb; i += 64) e[i] = ej[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += d[i];
    tot_d = s;
  }
  __syncthreads();
  if (!(tot_d > 0.0) || !isfinite(tot_d)) return;  // uniform decision: every thread returns
  for (int i = threadIdx.x; i < nb; i += 64) {
    double sm;
    if (nb == 1) sm = d[0];
    else if (i == 0) sm = 0.5 * (d[0] + d[1]);
    else if (i == nb - 1) sm = 0.5 * (d[nb - 2] + d[nb - 1]);
    else sm = (d[i - 1] + d[i] + d[i + 1]) / 3.0;
    r[i] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += r[i];
    tot_sm = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += 64) {
    const double p = r[i] / tot_sm;
    double v;
    if (p <= 0.0) v = 0.0;
    else if (p >= 1.0) v = 1.0;
    else v = pow((1.0 - p) / log(1.0 / p), alpha);
    r[i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    cum[0] = 0.0;
    for (int i = 0; i < nb; ++i) { s += r[i]; cum[i + 1] = s; }
  }
  __syncthreads();
  const double step = cum[nb] / (double)nb;
  for (int k = 1 + threadIdx.x; k < nb; k += 64) {
    const double target = (double)k * step;
    // smallest i in [0, nb-1) with cum[i+1] >= target, else nb-1
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cum[mid + 1] >= target) hi = mid; else lo = mid + 1;
    }
    const int i = lo;
    double frac = 0.0;
    if (r[i] > 0.0) {
      frac = (target - cum[i]) / r[i];
      frac = frac < 0.0 ? 0.0 : (frac > 1.0 ? 1.0 : frac);
    }
    ej[k] = e[i] + frac * (e[i + 1] - e[i]);
  }
}

}  // namespace vgx

struct vgx_vegas {
  int device = 0;
  hipStream_t stream = nullptr;
  int kind = 0, dim = 0, nb = 0, prec = 0;
  double alpha = 1.5;
  uint64_t seed = 0;
  uint32_t stream_id = 0;
  vgx::IntegrandParams prm{};
  vgx::TTbarConst tt{};
  vgx::DYConst dy{};
  vgx::STConst st{};
  vgx::TTDynConst ttd{};  // TTBAR mode 2 (scale set per event)
  int tt_dyn = 0;
  int max_wg = 0;
  int pstride = 0;
  double* edges = nullptr;          // [dim][nb+1]
  double* hist = nullptr;           // [dim][nb]
  double* partials = nullptr;       // [max_wg][pstride]
  float* tables = nullptr;          // the integrand's LDS tables, staged once (hadronic kinds)
  int table_bytes = 0;
  vgx::IterRecord* rec = nullptr;   // [MAX_RECORDS]
  vgx::Combined* comb = nullptr;
  void* pinned = nullptr;           // host readback (IterRecord + Combined + grid)
  int n_rec = 0;
  bool comb_fresh = false;           // the host copy of the combination (in pinned) is current
  int pend_k = -1;                  // record holding only S1, S2 until the next refinement completes it (< 0: none)
  int64_t pend_n = 0;               // its sample count
  double judge_var = -1.0;          // n var(E) of the latest plain iteration read back (< 0: none)
  bool have_hist = false;
  // kernel timing: event pairs recorded around the fused kernel, read back
  // (and summed) only when asked for, so timing does not synchronise
  static constexpr int kTimerPairs = 256;
  bool timing = false;
  int t_every = 1;                  // time one launch in t_every
  int64_t t_seen = 0;               // launches since timing was enabled
  hipEvent_t ev[2 * kTimerPairs] = {};
  int t_pending = 0;
  double t_ms = 0.0;
  int64_t t_launches = 0;
};

// Completes a record that vegas_iterate_async left pending (enqueued on the
// context's stream; nothing when none is pending).  Every path that reads
// the records or the combination, or adds a record, calls it first.
vgx_status vegas_flush_pending(vgx_vegas* v);
