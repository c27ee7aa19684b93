// Coupling-flow device code shared by the flow kernels and the fused
// flow-sampling VEGAS iteration: operand types, the layer descriptors,
// the network's tile products and the per-sample coupling transforms.
#pragma once

#include "common.h"

namespace vgx {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Operand precision of the networks' matrix products.  OpBF16 is the
// product path (v_mfma_f32_32x32x16_bf16).  OpF32 is a validation build of
// the same tile structure: a K = 16 step becomes eight K = 2 steps of
// v_mfma_f32_32x32x2_f32 over the same eight operand registers (lane (i, h)
// supplies k = h of step e, the element that the BF16 form reads as
// k = 8 h + e, so the sum over a step is the same), FP32 packs and tiles;
// with it the kernels can be compared with the FP64 oracle at FP32 rounding.
struct OpBF16 {
  using S = unsigned short;  // storage element of the weight packs and tiles
  using frag = bf16x8;
  static constexpr int kEs = 2;
  static __device__ __forceinline__ f32x16 mma(const frag& a, const frag& b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void set(frag& f, int e, float x) { f[e] = (__bf16)x; }
  static __device__ __forceinline__ float get(const frag& f, int e) { return (float)f[e]; }
  static __device__ __forceinline__ S store(float x) {
    const __bf16 b = (__bf16)x;
    return *(const S*)&b;
  }
};

struct OpF32 {
  using S = float;
  using frag = f32x8;
  static constexpr int kEs = 4;
  static __device__ __forceinline__ f32x16 mma(const frag& a, const frag& b, f32x16 c) {
#pragma unroll
    for (int e = 0; e < 8; ++e) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], c, 0, 0, 0);
    return c;
  }
  static __device__ __forceinline__ void set(frag& f, int e, float x) { f[e] = x; }
  static __device__ __forceinline__ float get(const frag& f, int e) { return f[e]; }
  static __device__ __forceinline__ S store(float x) { return x; }
};

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// ReLU, ReLU-derivative mask and element sum of an operand fragment.
template <class OP>
struct FragOps;

template <>
struct FragOps<OpBF16> {
  using frag = bf16x8;
  // a BF16 value is negative exactly when its bits are, read as a signed
  // 16-bit integer: max with 0 on packed pairs is the ReLU (v_pk_max_i16)
  static __device__ __forceinline__ void relu(frag& f) {
    const s16x8 x = __builtin_elementwise_max(__builtin_bit_cast(s16x8, f), (s16x8)0);
    f = __builtin_bit_cast(frag, x);
  }
  // d = (h > 0) ? d : 0 per element, for h >= 0 (a ReLU output): min(h, 1)
  // is 1 for every non-zero h and 0 for +0, and multiplies the bits of d
  static __device__ __forceinline__ void mask(frag& d, const frag& h) {
    u32x4v dv = __builtin_bit_cast(u32x4v, d);
    const u32x4v hv = __builtin_bit_cast(u32x4v, h);
    const unsigned one2 = 0x00010001u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      unsigned r;
      asm("v_pk_min_u16 %0, %1, %2\n\tv_pk_mul_lo_u16 %0, %3, %0" : "=&v"(r) : "v"(hv[k]), "v"(one2), "v"(dv[k]));
      dv[k] = r;
    }
    d = __builtin_bit_cast(frag, dv);
  }
  // acc + the sum of the eight elements (v_dot2 with ones)
  static __device__ __forceinline__ float sum(const frag& f, float acc) {
    const u32x4v v = __builtin_bit_cast(u32x4v, f);
    const bf16x2 one = {(__bf16)1.0f, (__bf16)1.0f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned w = v[k];
      acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, w), one, acc, false);
    }
    return acc;
  }
  // (whole vectors are bit_cast, then indexed: a bit_cast of one element
  // f[e] compiles to element 0)
  static __device__ __forceinline__ unsigned short bits(const frag& f, int e) {
    const u16x8 u = __builtin_bit_cast(u16x8, f);
    return u[e];
  }
};

template <>
struct FragOps<OpF32> {
  using frag = f32x8;
  static __device__ __forceinline__ void relu(frag& f) {
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = fmaxf(f[e], 0.0f);
  }
  static __device__ __forceinline__ void mask(frag& d, const frag& h) {
#pragma unroll
    for (int e = 0; e < 8; ++e) d[e] = h[e] > 0.0f ? d[e] : 0.0f;
  }
  static __device__ __forceinline__ float sum(const frag& f, float acc) {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc += f[e];
    return acc;
  }
  static __device__ __forceinline__ float bits(const frag& f, int e) { return f[e]; }
};

constexpr int FH = 64;       // hidden width
constexpr int FK = 32;       // bins
constexpr int FL_MAX = 8;    // layers
constexpr int FAB = 8;       // max |A|, |B|
constexpr int FDM = VGX_MAX_DIM;
constexpr int FBLOCK = 256;
constexpr int FWD_BLOCK = 512;  // forward kernels: 8 waves share one LDS copy of the weights

struct FlowLayerDesc {
  int na, nb;
  int a_idx[FAB], b_idx[FAB];
  int p_off;     // first parameter of the layer in the flat master vector
  int n_par;     // parameters of the layer
  int fw_off;    // bf16 offset of the layer's forward pack [W1p | W2p | W3p]
  int fw_len;
  int bw_off;    // bf16 offset of the layer's backward pack [W3Tp | W2Tp | W1Tp]
  int bw_len;
  int bias_off;  // float offset of [b1 | b2 | b3]
  int bias_len;
};

struct FlowDesc {
  int d, L;
  FlowLayerDesc l[FL_MAX];
  int fw_total, bw_total, bias_total;  // sizes of the packed buffers
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int v = 0; v < 16; ++v) z[v] = 0.0f;
  return z;
}

// 8 consecutive accumulator registers as a B operand (K step half 0 or 1).
template <class OP>
__device__ __forceinline__ typename OP::frag to_b(const f32x16& c, int half) {
  typename OP::frag r;
#pragma unroll
  for (int e = 0; e < 8; ++e) OP::set(r, e, half ? c[8 + e] : c[e]);
  return r;
}

// row (feature / bin) held by register v of lane half h in a 32x32 D tile
__device__ __forceinline__ int drow(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// value held by lane l ^ 32 of the wave: v_permlane32_swap trades the upper
// half of its first operand with the lower half of its second, so with both
// operands x the lower lanes find x[l + 32] in the second result and the
// upper lanes x[l - 32] in the first
__device__ __forceinline__ unsigned xor32u(unsigned x) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return (threadIdx.x & 32) ? r[0] : r[1];
}
__device__ __forceinline__ float xor32(float x) { return __uint_as_float(xor32u(__float_as_uint(x))); }
__device__ __forceinline__ int xor32i(int x) { return (int)xor32u((unsigned)x); }

// read / write z[j] for a runtime j without dynamic register indexing
__device__ __forceinline__ float zget(const float (&z)[FDM], int j) {
  float r = z[0];
#pragma unroll
  for (int k = 1; k < FDM; ++k) r = (k == j) ? z[k] : r;
  return r;
}
__device__ __forceinline__ void zset(float (&z)[FDM], int j, float v) {
#pragma unroll
  for (int k = 0; k < FDM; ++k) z[k] = (k == j) ? v : z[k];
}

template <class OP>
struct LayerLds {
  using frag = typename OP::frag;
  const frag* w1p;   // [2][32][2]
  const frag* w2p;   // [2][4][32][2]
  const frag* w3p;   // [nb][4][32][2]
  const float* b1;
  const float* b2;
  const float* b3;
};

template <class OP>
__device__ __forceinline__ LayerLds<OP> layer_lds(const typename OP::S* fw, const float* bias, const FlowLayerDesc& L,
                                                  int fw_base, int bias_base) {
  using frag = typename OP::frag;
  LayerLds<OP> r;
  const typename OP::S* p = fw + (L.fw_off - fw_base);
  r.w1p = (const frag*)p;
  r.w2p = (const frag*)(p + 1024);
  r.w3p = (const frag*)(p + 1024 + 4096);
  const float* b = bias + (L.bias_off - bias_base);
  r.b1 = b;
  r.b2 = b + FH;
  r.b3 = b + 2 * FH;
  return r;
}

// Accumulator tile holding bias b[row] in the register of each row of a
// 32x32 D tile (rows 8 (v >> 2) + 4 h + (v & 3)): four 16-byte LDS reads.
__device__ __forceinline__ f32x16 bias_tile(const float* b, int h) {
  f32x16 r;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4 q = *(const float4*)(b + 8 * g + 4 * h);
    r[4 * g] = q.x;
    r[4 * g + 1] = q.y;
    r[4 * g + 2] = q.z;
    r[4 * g + 3] = q.w;
  }
  return r;
}

// Network forward of one layer for the wave's 32 samples (transposed form);
// the biases enter as the accumulators' initial values.
template <int NBM, class OP>
__device__ __forceinline__ void mlp_fwd(const float (&za)[FAB], int na, int nb, const LayerLds<OP>& W, f32x16 (&h1)[2],
                                        f32x16 (&h2)[2], f32x16 (&lg)[NBM]) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  typename OP::frag bz;
#pragma unroll
  for (int e = 0; e < 8; ++e) OP::set(bz, e, (h == 0 && e < na) ? za[e] : 0.0f);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    h1[t] = OP::mma(W.w1p[(t * 32 + i) * 2 + h], bz, bias_tile(W.b1 + 32 * t, h));
#pragma unroll
    for (int v = 0; v < 16; ++v) h1[t][v] = fmaxf(h1[t][v], 0.0f);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x16 acc = bias_tile(W.b2 + 32 * t, h);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      acc = OP::mma(W.w2p[((t * 4 + kk) * 32 + i) * 2 + h], to_b<OP>(h1[kk >> 1], kk & 1), acc);
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = fmaxf(acc[v], 0.0f);
    h2[t] = acc;
  }
#pragma unroll
  for (int t = 0; t < NBM; ++t) {
    if (t < nb) {
      f32x16 acc = bias_tile(W.b3 + 32 * t, h);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        acc = OP::mma(W.w3p[((t * 4 + kk) * 32 + i) * 2 + h], to_b<OP>(h2[kk >> 1], kk & 1), acc);
      lg[t] = acc;
    }
  }
}

// The network's hidden layers for the wave's 32 samples (transposed form):
// h2 = relu(W2 relu(W1 zA + b1) + b2), returned as the four BF16 K-step
// operands of the output layer (each activation converted once).
template <class OP>
__device__ __forceinline__ void mlp_hidden(const float (&za)[FAB], int na, const LayerLds<OP>& W,
                                           typename OP::frag (&h2b)[4]) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  typename OP::frag bz;
#pragma unroll
  for (int e = 0; e < 8; ++e) OP::set(bz, e, (h == 0 && e < na) ? za[e] : 0.0f);
  typename OP::frag h1b[4];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const f32x16 p = OP::mma(W.w1p[(t * 32 + i) * 2 + h], bz, bias_tile(W.b1 + 32 * t, h));
    h1b[2 * t] = to_b<OP>(p, 0);
    h1b[2 * t + 1] = to_b<OP>(p, 1);
    FragOps<OP>::relu(h1b[2 * t]);
    FragOps<OP>::relu(h1b[2 * t + 1]);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x16 acc = bias_tile(W.b2 + 32 * t, h);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = OP::mma(W.w2p[((t * 4 + kk) * 32 + i) * 2 + h], h1b[kk], acc);
    h2b[2 * t] = to_b<OP>(acc, 0);
    h2b[2 * t + 1] = to_b<OP>(acc, 1);
    FragOps<OP>::relu(h2b[2 * t]);
    FragOps<OP>::relu(h2b[2 * t + 1]);
  }
}

// The 32 logits of transformed dimension t for the wave's 32 samples.
template <class OP>
__device__ __forceinline__ f32x16 mlp_logits(const typename OP::frag (&h2b)[4], int t, const LayerLds<OP>& W) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  f32x16 acc = bias_tile(W.b3 + 32 * t, h);
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = OP::mma(W.w3p[((t * 4 + kk) * 32 + i) * 2 + h], h2b[kk], acc);
  return acc;
}

// in place: exponentials of the 32 logits of one B dim less their maximum
// (16 here, 16 in lane^32), unnormalised; returns their sum
// e^(x - m) as 2^(x log2 e + nml) with nml = -m log2 e, on the hardware
// exp2 (v_exp_f32, relative error ~1e-7): the scale is folded into one FMA;
// the rounding of nml is common to all bins of a sample and cancels in the
// softmax's normalisation.
constexpr float FLOG2E = 1.44269504088896341f;
__device__ __forceinline__ float exp_shifted(float x, float nml) { return __builtin_amdgcn_exp2f(fmaf(x, FLOG2E, nml)); }

__device__ __forceinline__ float softexp32(f32x16& q) {
  float m = q[0];
#pragma unroll
  for (int v = 1; v < 16; ++v) m = fmaxf(m, q[v]);
  m = fmaxf(m, xor32(m));
  const float nml = -m * FLOG2E;
  float s = 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    q[v] = exp_shifted(q[v], nml);
    s += q[v];
  }
  return s + xor32(s);
}

// in-place softmax over the 32 bins of one B dim
__device__ __forceinline__ void softmax32(f32x16& q) {
  const float inv = 1.0f / softexp32(q);
#pragma unroll
  for (int v = 0; v < 16; ++v) q[v] *= inv;
}

// density direction for one B dim: returns z', sets the bin, alpha, Q_b;
// q holds the bin weights scaled by 1/inv (inv = 1 for probabilities)
__device__ __forceinline__ float cdf_fwd(const f32x16& q, float z, int& b, float& al, float& qb, float inv = 1.0f) {
  const int h = (threadIdx.x >> 5) & 1;
  const float t = z * (float)FK;
  int bb = (int)floorf(t);
  bb = bb < 0 ? 0 : (bb > FK - 1 ? FK - 1 : bb);
  al = t - (float)bb;
  float lt = 0.0f, qq = 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int k = drow(v, h);
    lt += (k < bb) ? q[v] : 0.0f;
    qq += (k == bb) ? q[v] : 0.0f;
  }
  lt = (lt + xor32(lt)) * inv;
  qq = (qq + xor32(qq)) * inv;
  b = bb;
  qb = qq;
  return lt + al * qq;
}

// sampling direction for one B dim: returns z, sets the bin and Q_b; q
// holds unnormalised bin weights with sum sum (the search runs on v sum)
__device__ __forceinline__ float cdf_inv(const f32x16& q, float v, float sum, int& b, float& qb) {
  v *= sum;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  float cs[4], ps[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) cs[g] = (q[4 * g] + q[4 * g + 1]) + (q[4 * g + 2] + q[4 * g + 3]);
#pragma unroll
  for (int g = 0; g < 4; ++g) ps[g] = xor32(cs[g]);
  // chunks c = 2g + h' hold bins 4c .. 4c+3; scan them in order
  float acc = 0.0f, base = 0.0f;
  int cstar = 7;
  bool found = false;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const float sc = ((c & 1) == h) ? cs[c >> 1] : ps[c >> 1];
    if (!found && (v < acc + sc || c == 7)) {
      found = true;
      cstar = c;
      base = acc;
    }
    acc += sc;
  }
  // the owner of chunk c* locates the bin inside it
  int bb = 4 * cstar + 3;
  float cb = base, qq = 0.0f;
  if ((cstar & 1) == h) {
    const int g = cstar >> 1;
    float run = base;
    bool got = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float qr = q[4 * g + r];
      if (!got && (v < run + qr || r == 3)) {
        got = true;
        bb = 4 * cstar + r;
        cb = run;
        qq = qr;
      }
      run += qr;
    }
  }
  // take the owner's values (own lane or lane ^ 32)
  const bool own = (cstar & 1) == h;
  const int bx = xor32i(bb);
  const float cx = xor32(cb), qx = xor32(qq);
  bb = own ? bb : bx;
  cb = own ? cb : cx;
  qq = own ? qq : qx;
  b = bb;
  qb = qq / sum;
  float frac = (v - cb) / qq;
  frac = frac < 0.0f ? 0.0f : (frac > 1.0f ? 1.0f : frac);
  return ((float)bb + frac) * (1.0f / (float)FK);
}

// copy n 16-byte chunks global -> LDS (whole workgroup)
__device__ __forceinline__ void copy16(void* dst, const void* src, int bytes) {
  const int4* s = (const int4*)src;
  int4* d = (int4*)dst;
  const int n = bytes / 16;
  int k = threadIdx.x;
  // 8 loads in flight per thread before their stores
  for (; k + 7 * (int)blockDim.x < n; k += 8 * blockDim.x) {
    int4 t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = s[k + q * blockDim.x];
#pragma unroll
    for (int q = 0; q < 8; ++q) d[k + q * blockDim.x] = t[q];
  }
  for (; k < n; k += blockDim.x) d[k] = s[k];
}

// ---------------------------------------------------------------------------
// Forward kernels: MODE 0 density (eval), 1 density (training), 2 sampling.
// ---------------------------------------------------------------------------
struct FwdArgs {
  int64_t n;
  const double* yin;    // density: [d][n]
  const double* g;      // training: [n]
  double* out;          // density: u [d][n] (nullable); sampling: y [d][n]
  double* logq;         // [n]
  float* zsave;         // training: [L][d][n]
  double* rsave;        // training: [n]
  double* partials;     // training: [grid][4]
  uint32_t it, sid, k0, k1;  // sampling: Philox counter / key
};

// LDS of a forward kernel: packed weights | biases | per-lane z [d][FWD_BLOCK]
// (es: bytes per packed weight)
__host__ __device__ inline size_t fwd_z_offset(int fw_total, int bias_total, int es) {
  return (((size_t)fw_total * es + (size_t)bias_total * 4) + 15) & ~(size_t)15;
}

// ---- one sample per lane after a tile pair's exchange ---------------------
// A wave runs the networks for two 32-sample tiles (samples 64 t + 0..31 and
// 64 t + 32..63); then one permlane32 swap per register of the two logit
// tiles gives every lane all 32 logits of its own sample 64 t + lane: bin
// k = 8 g + 4 hh + r sits in (hh ? hi : lo)[4 g + r].
__device__ __forceinline__ void pair_swap(f32x16& a, f32x16& b) {
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[v]), __float_as_uint(b[v]), false, false);
    a[v] = __uint_as_float(r[0]);
    b[v] = __uint_as_float(r[1]);
  }
}

// in place: exponentials of the lane's 32 logits less their maximum; returns
// their sum (unnormalised softmax)
__device__ __forceinline__ float softexp_own(f32x16& lo, f32x16& hi) {
  float m = fmaxf(lo[0], hi[0]);
#pragma unroll
  for (int v = 1; v < 16; ++v) m = fmaxf(m, fmaxf(lo[v], hi[v]));
  const float nml = -m * FLOG2E;
  float s = 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    lo[v] = exp_shifted(lo[v], nml);
    hi[v] = exp_shifted(hi[v], nml);
  }
  // bin-order sum in groups of four
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const f32x16& X = (c & 1) ? hi : lo;
    const int o = 4 * (c >> 1);
    s += (X[o] + X[o + 1]) + (X[o + 2] + X[o + 3]);
  }
  return s;
}

// the four weights of bin group c (bins 4c .. 4c+3) for a runtime c
__device__ __forceinline__ void group_vals(const f32x16& lo, const f32x16& hi, int c, float (&g)[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float v = lo[r];
#pragma unroll
    for (int cc = 1; cc < 8; ++cc) v = (c == cc) ? ((cc & 1) ? hi[4 * (cc >> 1) + r] : lo[4 * (cc >> 1) + r]) : v;
    g[r] = v;
  }
}

// density direction for one B dim of the lane's sample: returns z', sets
// the bin and Q_b; lo/hi hold the unnormalised bin weights, sum their sum
__device__ __forceinline__ float cdf_fwd_own(const f32x16& lo, const f32x16& hi, float sum, float z, int& b, float& qb) {
  const float t = z * (float)FK;
  int bb = (int)floorf(t);
  bb = bb < 0 ? 0 : (bb > FK - 1 ? FK - 1 : bb);
  const float al = t - (float)bb;
  const int cb = bb >> 2, rb = bb & 3;
  float lt = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const f32x16& X = (c & 1) ? hi : lo;
    const int o = 4 * (c >> 1);
    const float gsum = (X[o] + X[o + 1]) + (X[o + 2] + X[o + 3]);
    lt += (c < cb) ? gsum : 0.0f;
  }
  float g[4];
  group_vals(lo, hi, cb, g);
  float qq = g[0];
  lt += (rb > 0) ? g[0] : 0.0f;
  lt += (rb > 1) ? g[1] : 0.0f;
  lt += (rb > 2) ? g[2] : 0.0f;
  qq = (rb == 1) ? g[1] : qq;
  qq = (rb == 2) ? g[2] : qq;
  qq = (rb == 3) ? g[3] : qq;
  const float inv = 1.0f / sum;
  b = bb;
  qb = qq * inv;
  return lt * inv + al * qb;
}

// sampling direction for one B dim of the lane's sample: returns z, sets the
// bin and Q_b (search on v sum over the unnormalised cumulative weights)
__device__ __forceinline__ float cdf_inv_own(const f32x16& lo, const f32x16& hi, float sum, float v, int& b, float& qb) {
  const float vs = v * sum;
  float acc = 0.0f, base = 0.0f;
  int cstar = 7;
  bool found = false;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const f32x16& X = (c & 1) ? hi : lo;
    const int o = 4 * (c >> 1);
    const float gsum = (X[o] + X[o + 1]) + (X[o + 2] + X[o + 3]);
    const bool here = !found && (vs < acc + gsum || c == 7);
    cstar = here ? c : cstar;
    base = here ? acc : base;
    found = found || here;
    acc += gsum;
  }
  float g[4];
  group_vals(lo, hi, cstar, g);
  int bb = 4 * cstar + 3;
  float cb = base, qq = g[3], run = base;
  bool got = false;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const bool here = !got && (vs < run + g[r] || r == 3);
    bb = here ? 4 * cstar + r : bb;
    cb = here ? run : cb;
    qq = here ? g[r] : qq;
    got = got || here;
    run += g[r];
  }
  b = bb;
  qb = qq / sum;
  float frac = (vs - cb) / qq;
  frac = frac < 0.0f ? 0.0f : (frac > 1.0f ? 1.0f : frac);
  return ((float)bb + frac) * (1.0f / (float)FK);
}

// Draw the lane's sample i of a flow-sampling pass: coordinates u from
// Philox (counter (i, it, sid << 8 | block), key (k0, k1)) into the lane's
// z column (stride BS, the workgroup's threads).
template <int BS = FWD_BLOCK>
__device__ __forceinline__ void flow_draw(float* z, int d, int64_t i, uint32_t it, uint32_t sid, uint32_t k0,
                                          uint32_t k1) {
  for (int bk = 0; 4 * bk < d; ++bk) {
    const u32x4 w = philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), it, (sid << 8) | (uint32_t)bk, k0, k1);
    const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (4 * bk + e < d) z[(4 * bk + e) * BS] = (float)word_to_unit(ww[e]);
  }
}

// The coupling layers for the wave's tile pair (samples 64 t + lane): the
// lane's sample is in its own z column (stride BS); density direction
// (SAMPLING false, layers 0 .. L-1) or sampling direction (true, layers
// L-1 .. 0).  Returns log q; with zsave (density direction), each layer's
// input is saved to zsave [L][d][n] for valid samples.  Every lane of the
// wave must call it (cross-lane exchanges).
template <bool SAMPLING, class OP, int BS = FWD_BLOCK>
__device__ __forceinline__ double flow_layers(const FlowDesc& D, const typename OP::S* sfw, const float* sb, float* z,
                                              int64_t i, bool valid, float* zsave, int64_t n) {
  const int d = D.d;
  double lq = 0.0;
  for (int step = 0; step < D.L; ++step) {
    const int l = SAMPLING ? D.L - 1 - step : step;
    const FlowLayerDesc& L = D.l[l];
    if (!SAMPLING && zsave && valid) {
      for (int j = 0; j < d; ++j) zsave[((int64_t)l * d + j) * n + i] = z[j * BS];
    }
    // network inputs: tile A (samples 64 t + 0..31) takes the lower lanes'
    // own coordinates, tile B (64 t + 32..63) the upper lanes', moved down
    float za[FAB], zb[FAB];
#pragma unroll
    for (int e = 0; e < FAB; ++e) {
      za[e] = (e < L.na) ? z[L.a_idx[e] * BS] : 0.0f;
      zb[e] = xor32(za[e]);
    }
    const LayerLds<OP> W = layer_lds<OP>(sfw, sb, L, 0, 0);
    typename OP::frag h2A[4], h2B[4];
    mlp_hidden<OP>(za, L.na, W, h2A);
    mlp_hidden<OP>(zb, L.na, W, h2B);
    // one transformed dimension at a time: its logits for both tiles,
    // exchanged so that every lane holds its own sample's 32 logits
    for (int jb = 0; jb < L.nb; ++jb) {
      f32x16 lo = mlp_logits<OP>(h2A, jb, W), hi = mlp_logits<OP>(h2B, jb, W);
      pair_swap(lo, hi);
      const float sum = softexp_own(lo, hi);
      const int j = L.b_idx[jb];
      const float zj = z[j * BS];
      int b;
      float qb;
      const float zn = SAMPLING ? cdf_inv_own(lo, hi, sum, zj, b, qb) : cdf_fwd_own(lo, hi, sum, zj, b, qb);
      z[j * BS] = zn;
      lq += (double)logf((float)FK * qb);
    }
  }
  return lq;
}

// What the fused flow-sampling VEGAS iteration needs of a flow.
struct FlowView {
  const FlowDesc* desc;  // device copy of the layer descriptors
  const void* fw;        // forward packs (OpBF16::S or OpF32::S elements)
  const float* bias;
  int fw_total, bias_total, dim, L, nbm, f32ops;
};

}  // namespace vgx

struct vgx_flow;
namespace vgx {
FlowView flow_view(const vgx_flow* f);
// make stream s wait for the work enqueued on the flow's stream so far
vgx_status flow_order_before(vgx_flow* f, hipStream_t s);
}  // namespace vgx
