// Coupling-flow proposal (neural importance sampling) on MFMA: sampling,
// density, loss gradient and Adam.
//
// The thesis has no normalizing flow.  It gives the importance-sampling
// estimator and its variance (MC chapter), the dense layer y = phi(W x + b)
// and the activation table (deep-learning chapter), the training loop and
// the Adam equations (optimiser section).  The coupling transform is the
// piecewise-linear one of Mueller et al. (2019).  Per layer l the dims B_l
// are transformed conditioned on the others A_l through a network
// |A| -> 64 -> 64 -> |B| 32 (ReLU), softmax over 32 bins per B dim:
//   density  direction: b = floor(32 z), z' = C_b + (32 z - b) Q_b,
//   sampling direction: the inverse, b with C_b <= v < C_{b+1},
//   log q += ln(32 Q_b) in both.
// Loss: L = mean(g^2/q)/mean(g^2) on uniform points y of the VEGAS cube.
//
// MI355X design
//   * one wave handles a tile of 32 samples; every matrix product of the
//     networks runs on v_mfma_f32_32x32x16_bf16 in the transposed form
//     (features x samples), BF16 operands, FP32 accumulation;
//   * the D-layout of one product is fed to the next as the B operand
//     without shuffles: 8 consecutive accumulator registers form one K=16
//     step whose K order is a fixed permutation of the features, and the
//     weights are packed once (after every Adam step) in that permuted
//     order, so each A fragment is one 16-byte LDS read;
//   * the 32 bin probabilities of a B dim for one sample sit in 2 lanes
//     (l, l^32); softmax, cumulative sums and bin searches need one
//     cross-lane exchange each;
//   * training: a forward kernel (all layers, weights in LDS) saves each
//     layer's input; per layer (last to first) a backward kernel recomputes
//     the network, back-propagates to the layer input and writes BF16
//     operand tiles, and a weight-gradient kernel reduces them with MFMA
//     over the samples; one kernel reduces the per-workgroup partials in a
//     fixed order and applies Adam to the FP32 master weights; log-
//     densities and loss sums are FP64.
#include "common.h"
#include "flow_internal.h"

#include <algorithm>
#include <math.h>
#include <stdlib.h>
#include <vector>

namespace vgx {

template <int NBM, int MODE, class OP>
__global__ __launch_bounds__(FWD_BLOCK) void k_flow_fwd(const FlowDesc* __restrict__ Dp, FwdArgs a,
                                                     const typename OP::S* __restrict__ fw,
                                                     const float* __restrict__ bias) {
  using S = typename OP::S;
  extern __shared__ __align__(16) unsigned char flds[];
  const FlowDesc& D = *Dp;
  S* sfw = (S*)flds;
  float* sb = (float*)(flds + (size_t)D.fw_total * sizeof(S));
  // each lane keeps its own sample's coordinates in its own LDS column (the
  // layer masks index them with runtime, wave-uniform indices)
  float* z = (float*)(flds + fwd_z_offset(D.fw_total, D.bias_total, (int)sizeof(S))) + threadIdx.x;
  copy16(sfw, fw, D.fw_total * (int)sizeof(S));
  copy16(sb, bias, D.bias_total * 4);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = (threadIdx.x >> 6) * gridDim.x + blockIdx.x;
  const int nwaves = gridDim.x * (FWD_BLOCK / 64);
  const int64_t ntiles = (a.n + 63) / 64;  // tile pairs
  const int d = D.d;
  Comp sr, sg;
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    const int64_t i = t * 64 + lane;  // the lane's own sample
    const bool valid = i < a.n;
    if (MODE == 2) {
      flow_draw(z, d, i, a.it, a.sid, a.k0, a.k1);
    } else {
      for (int j = 0; j < d; ++j) z[j * FWD_BLOCK] = valid ? (float)a.yin[(int64_t)j * a.n + i] : 0.5f;
    }
    const double lq = flow_layers<MODE == 2, OP>(D, sfw, sb, z, i, valid, MODE == 1 ? a.zsave : nullptr, a.n);
    if (valid) {
      a.logq[i] = lq;
      if (a.out) {
        for (int j = 0; j < d; ++j) a.out[(int64_t)j * a.n + i] = (double)z[j * FWD_BLOCK];
      }
      if (MODE == 1) {
        const double gi = a.g[i];
        const double r = gi * gi * exp(-lq);
        a.rsave[i] = r;
        sr.add(r);
        sg.add(gi * gi);
      }
    }
  }
  if (MODE == 1) {
    __shared__ double red[4][FWD_BLOCK / 64];
    const double v0 = wave_sum(sr.s), v1 = wave_sum(sr.c), v2 = wave_sum(sg.s), v3 = wave_sum(sg.c);
    const int wv = threadIdx.x >> 6;
    if (lane == 0) { red[0][wv] = v0; red[1][wv] = v1; red[2][wv] = v2; red[3][wv] = v3; }
    __syncthreads();
    if (threadIdx.x < 4) {
      double acc = 0.0;
      for (int k = 0; k < FWD_BLOCK / 64; ++k) acc += red[threadIdx.x][k];
      a.partials[blockIdx.x * 4 + threadIdx.x] = acc;
    }
  }
}

// loss L = sum r / sum g^2, scale = -1/sum g^2 and the ok flag from the
// forward's partial rows [rows][4], by one wave (every lane gets them):
// lane l sums rows l, l + 64, ... (compensated), then the lanes combine in a
// fixed butterfly order and lane 0's totals are broadcast.  The loads of the
// first 512 rows are issued apart (loss_load), so that other work can run
// while they are in flight.
struct LossRows {
  double v[8][4];
};

__device__ __forceinline__ void loss_load(const double* __restrict__ partials, int rows, int r0, LossRows& lr) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int r = r0 + 64 * k + lane;
#pragma unroll
    for (int col = 0; col < 4; ++col) lr.v[k][col] = r < rows ? partials[r * 4 + col] : 0.0;
  }
}

__device__ __forceinline__ void loss_finish(const double* __restrict__ partials, int rows, LossRows& lr,
                                            double (&out)[3]) {
  const int lane = threadIdx.x & 63;
  Comp c[4];
  for (int r0 = 0; r0 < rows; r0 += 8 * 64) {
    if (r0 > 0) loss_load(partials, rows, r0, lr);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (r0 + 64 * k + lane < rows) {
#pragma unroll
        for (int col = 0; col < 4; ++col) c[col].add(lr.v[k][col]);
      }
  }
  double tot[4];
#pragma unroll
  for (int col = 0; col < 4; ++col) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double os = __shfl_xor(c[col].s, off, 64), oc = __shfl_xor(c[col].c, off, 64);
      c[col].add(os);
      c[col].add(oc);
    }
    tot[col] = __shfl(c[col].value(), 0, 64);
  }
  const double sr = tot[0] + tot[1], sg = tot[2] + tot[3];
  const double L = sr / sg;
  out[0] = L;
  out[1] = -1.0 / sg;
  out[2] = (isfinite(L) && sg > 0.0) ? 1.0 : 0.0;
}

__device__ __forceinline__ void loss_reduce(const double* __restrict__ partials, int rows, double (&out)[3]) {
  LossRows lr;
  loss_load(partials, rows, 0, lr);
  loss_finish(partials, rows, lr, out);
}

__global__ __launch_bounds__(64) void k_flow_loss(const double* __restrict__ partials, int rows, double* __restrict__ out) {
  double v[3];
  loss_reduce(partials, rows, v);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
  }
}

// ---------------------------------------------------------------------------
// Backward of one layer (data gradients + BF16 operand tiles for dW).
// Scratch rows per 32-sample tile: [zA 32][h1 64][h2 64][dpre1 64][dpre2 64][dlogit 32 nb].
// ---------------------------------------------------------------------------
struct BwdArgs {
  int64_t n;
  int layer;
  const float* zin;     // [d][n] input of this layer (saved by the forward)
  const float* dzout;   // [d][n] gradient w.r.t. the layer output (null: zero)
  float* dzin;          // [d][n] gradient w.r.t. the layer input
  const double* rsave;  // [n]
  const double* loss;   // [3]: L, scale, ok
  void* scr;            // operand tiles (OP::S elements)
  int srows;            // scratch rows per tile
  const double* partials;  // fused kernel: the forward's partial rows [prows][4], or null (loss read
  int prows;               // from loss); with them every workgroup reduces the loss itself and
  double* loss_out;        // workgroup 0 stores it to loss_out [3]
};

template <class OP>
__device__ __forceinline__ void put_tile(typename OP::S* base, int row0, const f32x16& c, int s, int h) {
#pragma unroll
  for (int v = 0; v < 16; ++v) base[(row0 + drow(v, h)) * 32 + s] = OP::store(c[v]);
}

// LDS of the backward kernel: the layer's forward and backward packs and
// biases, then per-lane columns z, dz_out, dz [3][d][FBLOCK]
__host__ __device__ inline size_t bwd_z_offset(int fw_len, int bw_len, int bias_len, int es) {
  return (((size_t)fw_len * es + (size_t)bw_len * es + (size_t)bias_len * 4) + 15) & ~(size_t)15;
}

template <int NBM, class OP>
__global__ __launch_bounds__(FBLOCK, (NBM <= 2 ? 2 : 1)) void k_flow_bwd(const FlowDesc* __restrict__ Dp, BwdArgs a,
                                                                       const typename OP::S* __restrict__ fw,
                                                                       const typename OP::S* __restrict__ bw,
                                                                       const float* __restrict__ bias) {
  using S = typename OP::S;
  using frag = typename OP::frag;
  extern __shared__ __align__(16) unsigned char flds[];
  const FlowDesc& D = *Dp;
  const FlowLayerDesc& L = D.l[a.layer];
  S* sfw = (S*)flds;
  S* sbw = sfw + L.fw_len;
  float* sb = (float*)(sbw + L.bw_len);
  const int d = D.d;
  // the sample's coordinates (z), the incoming gradient (gz) and the
  // outgoing gradient (dz) in the lane's own LDS columns
  float* z = (float*)(flds + bwd_z_offset(L.fw_len, L.bw_len, L.bias_len, (int)sizeof(S))) + threadIdx.x;
  float* gz = z + d * FBLOCK;
  float* dz = gz + d * FBLOCK;
  copy16(sfw, fw + L.fw_off, L.fw_len * (int)sizeof(S));
  copy16(sbw, bw + L.bw_off, L.bw_len * (int)sizeof(S));
  copy16(sb, bias + L.bias_off, L.bias_len * 4);
  __syncthreads();
  const LayerLds<OP> W = layer_lds<OP>(sfw, sb, L, L.fw_off, L.bias_off);
  const frag* w3t = (const frag*)sbw;                         // [2][2nb][32][2]
  const frag* w2t = (const frag*)(sbw + L.nb * 2048);         // [2][4][32][2]
  const frag* w1t = (const frag*)(sbw + L.nb * 2048 + 4096);  // [1][4][32][2]
  const double scale = a.loss[1];
  const int lane = threadIdx.x & 63, s = lane & 31, h = lane >> 5;
  const int wave = blockIdx.x * (FBLOCK / 64) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (FBLOCK / 64);
  const int64_t ntiles = (a.n + 31) / 32;
  const int na = L.na, nb = L.nb;
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    const int64_t i = t * 32 + s;
    const bool valid = i < a.n;
    for (int j = 0; j < d; ++j) {
      z[j * FBLOCK] = valid ? a.zin[(int64_t)j * a.n + i] : 0.5f;
      const float g0 = (valid && a.dzout) ? a.dzout[(int64_t)j * a.n + i] : 0.0f;
      gz[j * FBLOCK] = g0;
      dz[j * FBLOCK] = g0;
    }
    const float dlq = valid ? (float)(a.rsave[i] * scale) : 0.0f;
    float za[FAB];
#pragma unroll
    for (int e = 0; e < FAB; ++e) za[e] = (e < na) ? z[L.a_idx[e] * FBLOCK] : 0.0f;
    f32x16 h1[2], h2[2], lg[NBM];
    mlp_fwd<NBM, OP>(za, na, nb, W, h1, h2, lg);
    // operand tiles for the weight gradients, written as soon as they
    // exist; only the ReLU masks of h1, h2 stay live (invalid samples carry
    // zero deltas, so they add nothing)
    S* base = (S*)a.scr + (size_t)t * a.srows * 32;
#pragma unroll
    for (int e = 0; e < 8; ++e) base[(8 * h + e) * 32 + s] = OP::store((h == 0 && e < na) ? za[e] : 0.0f);
    put_tile<OP>(base, 32, h1[0], s, h);
    put_tile<OP>(base, 64, h1[1], s, h);
    put_tile<OP>(base, 96, h2[0], s, h);
    put_tile<OP>(base, 128, h2[1], s, h);
    unsigned m1[2] = {0u, 0u}, m2[2] = {0u, 0u};
#pragma unroll
    for (int to = 0; to < 2; ++to)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        m1[to] |= (h1[to][v] > 0.0f ? 1u : 0u) << v;
        m2[to] |= (h2[to][v] > 0.0f ? 1u : 0u) << v;
      }
    // bins, dQ and dlogit per transformed dim
#pragma unroll
    for (int jb = 0; jb < NBM; ++jb) {
      if (jb < nb) {
        softmax32(lg[jb]);
        const int j = L.b_idx[jb];
        int b;
        float al, qb;
        cdf_fwd(lg[jb], z[j * FBLOCK], b, al, qb);
        const float g_out = gz[j * FBLOCK];
        float dq[16];
        float sdot = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int k = drow(v, h);
          dq[v] = g_out * ((k < b) ? 1.0f : ((k == b) ? al : 0.0f)) + ((k == b) ? dlq / qb : 0.0f);
          sdot += lg[jb][v] * dq[v];
        }
        sdot += xor32(sdot);
#pragma unroll
        for (int v = 0; v < 16; ++v) lg[jb][v] = lg[jb][v] * (dq[v] - sdot);  // dlogit
        dz[j * FBLOCK] = g_out * (float)FK * qb;
        put_tile<OP>(base, 288 + 32 * jb, lg[jb], s, h);
      }
    }
    // dh2 = W3^T dlogit, masked by relu'
    f32x16 d2[2];
#pragma unroll
    for (int to = 0; to < 2; ++to) {
      f32x16 acc = zero16();
#pragma unroll
      for (int kk = 0; kk < 2 * NBM; ++kk)
        if (kk < 2 * nb) acc = OP::mma(w3t[((to * 2 * nb + kk) * 32 + s) * 2 + h], to_b<OP>(lg[kk >> 1], kk & 1), acc);
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = ((m2[to] >> v) & 1u) ? acc[v] : 0.0f;
      d2[to] = acc;
    }
    put_tile<OP>(base, 224, d2[0], s, h);
    put_tile<OP>(base, 256, d2[1], s, h);
    // dh1 = W2^T dpre2, masked
    f32x16 d1[2];
#pragma unroll
    for (int to = 0; to < 2; ++to) {
      f32x16 acc = zero16();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = OP::mma(w2t[((to * 4 + kk) * 32 + s) * 2 + h], to_b<OP>(d2[kk >> 1], kk & 1), acc);
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = ((m1[to] >> v) & 1u) ? acc[v] : 0.0f;
      d1[to] = acc;
    }
    put_tile<OP>(base, 160, d1[0], s, h);
    put_tile<OP>(base, 192, d1[1], s, h);
    // dzA = W1^T dpre1: rows a = 4h + r in registers 0..3
    f32x16 d0 = zero16();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) d0 = OP::mma(w1t[(kk * 32 + s) * 2 + h], to_b<OP>(d1[kk >> 1], kk & 1), d0);
    float dza[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float mine = d0[r], other = xor32(d0[r]);
      dza[r] = h == 0 ? mine : other;
      dza[4 + r] = h == 0 ? other : mine;
    }
#pragma unroll
    for (int e = 0; e < FAB; ++e)
      if (e < na) dz[L.a_idx[e] * FBLOCK] += dza[e];
    if (valid && h == 0) {
      for (int j = 0; j < d; ++j) a.dzin[(int64_t)j * a.n + i] = dz[j * FBLOCK];
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradients of one layer: dW3 = dlogit h2^T, dW2 = dpre2 h1^T,
// dW1 = dpre1 zA^T (K = samples, MFMA), biases = row sums of the deltas.
// Each workgroup writes its partial of the layer's parameter block.
// ---------------------------------------------------------------------------
struct WgradArgs {
  int64_t n;
  int layer;
  const void* scr;  // operand tiles (OP::S elements)
  int srows;
  float* gpart;   // [grid][n_par] partials of this layer
};

template <class OP>
__device__ __forceinline__ typename OP::frag ld_frag(const typename OP::S* base, int row, int kk, int h) {
  return *(const typename OP::frag*)(base + row * 32 + 16 * kk + 8 * h);
}

template <class OP>
__device__ __forceinline__ float frag_sum(const typename OP::frag& x) {
  float s = 0.0f;
#pragma unroll
  for (int e = 0; e < 8; ++e) s += OP::get(x, e);
  return s;
}

template <int MT, int NT, class OP>
__device__ __forceinline__ void wgrad_gemm(const typename OP::S* scr, int srows, int64_t ntiles, int wave, int nwaves,
                                           int arow0, int brow0, int mt, int nt, f32x16 (&acc)[MT][NT],
                                           float (&bsum)[MT]) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    bsum[m] = 0.0f;
#pragma unroll
    for (int nn = 0; nn < NT; ++nn) acc[m][nn] = zero16();
  }
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    const typename OP::S* base = scr + (size_t)t * srows * 32;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      typename OP::frag bf[NT];
#pragma unroll
      for (int nn = 0; nn < NT; ++nn)
        if (nn < nt) bf[nn] = ld_frag<OP>(base, brow0 + 32 * nn + i, kk, h);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        if (m < mt) {
          const typename OP::frag af = ld_frag<OP>(base, arow0 + 32 * m + i, kk, h);
          bsum[m] += frag_sum<OP>(af);
#pragma unroll
          for (int nn = 0; nn < NT; ++nn)
            if (nn < nt) acc[m][nn] = OP::mma(af, bf[nn], acc[m][nn]);
        }
      }
    }
  }
}

// add a D tile (rows = output rows of W, cols = input columns) into the LDS
// parameter block W[row][col] with row stride ld, columns < ncol only; plain
// adds: the caller lets one wave at a time do this (in_wave_order)
__device__ __forceinline__ void add_tile(float* blk, int ld, int row0, int col0, int ncol, const f32x16& c) {
  const int lane = threadIdx.x & 63, j = lane & 31, h = lane >> 5;
  if (col0 + j < ncol) {
#pragma unroll
    for (int v = 0; v < 16; ++v) blk[(row0 + drow(v, h)) * ld + col0 + j] += c[v];
  }
}

// Run f() in each wave of the workgroup in turn, wave 0 first: the waves'
// contributions meet in the LDS block in a fixed order and without atomics
// (LDS float atomics from four waves measured 31 us of a 51 us launch).
template <class Fn>
__device__ __forceinline__ void in_wave_order(Fn&& f) {
  const int w = threadIdx.x >> 6;
  for (int k = 0; k < FBLOCK / 64; ++k) {
    if (w == k) f();
    __syncthreads();
  }
}

template <int NBM, class OP>
__global__ __launch_bounds__(FBLOCK) void k_flow_wgrad(const FlowDesc* __restrict__ Dp, WgradArgs a) {
  const typename OP::S* scr = (const typename OP::S*)a.scr;
  extern __shared__ __align__(16) unsigned char flds[];
  const FlowLayerDesc& L = Dp->l[a.layer];
  float* blk = (float*)flds;  // the layer's parameter block
  for (int k = threadIdx.x; k < L.n_par; k += FBLOCK) blk[k] = 0.0f;
  __syncthreads();
  const int na = L.na, nb = L.nb;
  const int oW1 = 0, ob1 = FH * na, oW2 = ob1 + FH, ob2 = oW2 + FH * FH, oW3 = ob2 + FH, ob3 = oW3 + nb * FK * FH;
  const int wave = blockIdx.x * (FBLOCK / 64) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (FBLOCK / 64);
  const int64_t ntiles = (a.n + 31) / 32;
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  {  // dW3 [o][f], db3
    f32x16 acc[NBM][2];
    float bs[NBM];
    wgrad_gemm<NBM, 2, OP>(scr, a.srows, ntiles, wave, nwaves, 288, 96, nb, 2, acc, bs);
    in_wave_order([&] {
#pragma unroll
      for (int m = 0; m < NBM; ++m)
        if (m < nb) {
#pragma unroll
          for (int nn = 0; nn < 2; ++nn) add_tile(blk + oW3, FH, 32 * m, 32 * nn, FH, acc[m][nn]);
          const float tot = bs[m] + xor32(bs[m]);
          if (h == 0) blk[ob3 + 32 * m + i] += tot;
        }
    });
  }
  {  // dW2 [f][f'], db2
    f32x16 acc[2][2];
    float bs[2];
    wgrad_gemm<2, 2, OP>(scr, a.srows, ntiles, wave, nwaves, 224, 32, 2, 2, acc, bs);
    in_wave_order([&] {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
#pragma unroll
        for (int nn = 0; nn < 2; ++nn) add_tile(blk + oW2, FH, 32 * m, 32 * nn, FH, acc[m][nn]);
        const float tot = bs[m] + xor32(bs[m]);
        if (h == 0) blk[ob2 + 32 * m + i] += tot;
      }
    });
  }
  {  // dW1 [f][a], db1
    f32x16 acc[2][1];
    float bs[2];
    wgrad_gemm<2, 1, OP>(scr, a.srows, ntiles, wave, nwaves, 160, 0, 2, 1, acc, bs);
    in_wave_order([&] {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        add_tile(blk + oW1, na, 32 * m, 0, na, acc[m][0]);
        const float tot = bs[m] + xor32(bs[m]);
        if (h == 0) blk[ob1 + 32 * m + i] += tot;
      }
    });
  }
  float* out = a.gpart + (size_t)blockIdx.x * L.n_par;
  for (int k = threadIdx.x; k < L.n_par; k += FBLOCK) out[k] = blk[k];
}

// ---------------------------------------------------------------------------
// Fused backward and weight gradients of one layer (|B| <= 4).
//
// The workgroup's WV waves (8 where the stages fit the LDS, two per SIMD,
// else 4) take WV 32-sample tiles at a time (a group).  Each wave runs the
// backward of its tile as k_flow_bwd does; the operands
// of the weight-gradient products (deltas and activations, feature-major)
// go to an LDS stage instead of global memory, one product at a time:
// [dlogit | h2], then [dpre2 | h1], then [dpre1 | zA].  After each stage the
// waves contract the group's tiles (K = 32 WV samples) into the
// weight-gradient tiles they own: output tile tau of [dW3 (2 |B|) | dW2 (4) |
// dW1 (2)] belongs to wave tau mod WV, whose accumulators persist over all
// the tiles of the workgroup.  Each workgroup finally stores its partial of
// the layer's parameter block (every element from its one owner: no LDS
// reduction), in the layout k_flow_wgrad writes.  The next group's inputs
// are loaded while the current one is processed.  |B| is a template
// parameter, and the layer's coordinate sets are addressed through per-lane
// LDS pointers set up once, so the loop over groups has no branches on the
// layer's shape and reads nothing from its descriptor.
//
// Activations and deltas between the products stay in operand form (eight
// BF16 values per fragment): the ReLU, its derivative's mask and the bias
// sums work on packed pairs.
// ---------------------------------------------------------------------------
constexpr int FUSE_DMAX = 8;  // |B| <= 4 holds exactly for d <= 8

// rows of a tile's stage: the largest of (32 |B| + 64), 128 and 96
__host__ __device__ constexpr int fuse_stage_rows(int nb) { return 32 * nb + 64 > 128 ? 32 * nb + 64 : 128; }
// row stride of a stage in elements: 32 samples, + 16 bytes of padding for
// BF16 stages (the FP32 validation stages go without, to fit the LDS)
template <class OP>
__host__ __device__ constexpr int fuse_rs() { return sizeof(typename OP::S) == 2 ? 40 : 32; }

// LDS of the fused kernel with bs threads: packs and biases | per-lane
// columns [2 d + 2][bs] (z, its gradient, a zero column, a sink column) |
// stage [bs / 64][rows][rs]
__host__ __device__ inline size_t fuse_z_offset(int fw_len, int bw_len, int bias_len, int es) {
  return bwd_z_offset(fw_len, bw_len, bias_len, es);
}
__host__ __device__ inline size_t fuse_stage_offset(int fw_len, int bw_len, int bias_len, int es, int d, int bs) {
  return fuse_z_offset(fw_len, bw_len, bias_len, es) + sizeof(float) * (2 * (size_t)d + 2) * bs;
}

// the two hidden layers of the network for the wave's 32 samples as operand
// fragments (ReLU applied): h1b for the second product, h2b for the output;
// za holds zeros beyond |A|
template <class OP>
__device__ __forceinline__ void mlp_hidden_fb(const float (&za)[FAB], const LayerLds<OP>& W, typename OP::frag (&h1b)[4],
                                              typename OP::frag (&h2b)[4]) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  typename OP::frag bz;
#pragma unroll
  for (int e = 0; e < 8; ++e) OP::set(bz, e, h == 0 ? za[e] : 0.0f);
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

// fragment kk of a 32-row block into a stage, feature-major (row = feature,
// column = sample): element e holds row row0 + drow(8 (kk & 1) + e, h)
template <class OP>
__device__ __forceinline__ void stage_put(typename OP::S* st, int row0, const typename OP::frag& f, int half, int s,
                                          int h) {
  constexpr int RS = fuse_rs<OP>();
#pragma unroll
  for (int e = 0; e < 8; ++e) st[(row0 + drow(8 * half + e, h)) * RS + s] = FragOps<OP>::bits(f, e);
}

template <class OP>
__device__ __forceinline__ typename OP::frag stage_get(const typename OP::S* st, int row, int kk, int h) {
  constexpr int RS = fuse_rs<OP>();
  return *(const typename OP::frag*)(st + row * RS + 16 * kk + 8 * h);
}

// contract the group's NST stages: A rows arow0 + 32 m, B rows brow0 + 32 n
template <class OP, int NST, int SR>
__device__ __forceinline__ void fuse_contract(const typename OP::S* stage, int arow0, int brow0, int m, int n,
                                              f32x16& acc, float& bsum) {
  constexpr int RS = fuse_rs<OP>();
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
#pragma unroll
  for (int q = 0; q < NST; ++q) {
    const typename OP::S* st = stage + (size_t)q * SR * RS;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const typename OP::frag af = stage_get<OP>(st, arow0 + 32 * m + i, kk, h);
      const typename OP::frag bf = stage_get<OP>(st, brow0 + 32 * n + i, kk, h);
      if (n == 0) bsum = FragOps<OP>::sum(af, bsum);
      acc = OP::mma(af, bf, acc);
    }
  }
}

template <int NB, int WV, class OP>
__global__ __launch_bounds__(64 * WV) void k_flow_bwdw(const FlowDesc* __restrict__ Dp, BwdArgs a,
                                                     const typename OP::S* __restrict__ fw,
                                                     const typename OP::S* __restrict__ bw,
                                                     const float* __restrict__ bias, float* __restrict__ gpart) {
  static_assert(NB >= 1 && NB <= 4, "the fused kernel holds at most four weight-gradient tiles per wave");
  using S = typename OP::S;
  using frag = typename OP::frag;
  using FO = FragOps<OP>;
  constexpr int SR = fuse_stage_rows(NB);
  constexpr int RS = fuse_rs<OP>();
  constexpr int BS = 64 * WV;
  constexpr int T3 = 2 * NB, T = 2 * NB + 6;
  constexpr int OWN = (T + WV - 1) / WV;  // output tiles per wave
  extern __shared__ __align__(16) unsigned char flds[];
  const FlowDesc& D = *Dp;
  const FlowLayerDesc& L = D.l[a.layer];
  const int d = D.d;
  const int es = (int)sizeof(S);
  const int lane = threadIdx.x & 63, s = lane & 31, h = lane >> 5;
  const int wave = threadIdx.x >> 6;
  const int64_t n = a.n;
  const int64_t ntiles = (n + 31) / 32;
  const int64_t ngroups = (ntiles + WV - 1) / WV;
  // the inputs of the wave's tile of group g: coordinates z, incoming
  // gradient, the sample's loss term; a tile past the end has no valid
  // sample: zero deltas, nothing added.  Every load reads a valid address
  // (coordinates j >= d repeat d - 1, samples past the end read sample 0).
  const float* dzsrc = a.dzout ? a.dzout : a.zin;
  const float dzs = a.dzout ? 1.0f : 0.0f;
  float pz[FUSE_DMAX], pd[FUSE_DMAX];
  double pr;
  auto fetch = [&](int64_t g) {
    const int64_t i = (g * WV + wave) * 32 + s;
    const bool ok = g < ngroups && i < n;
    const int64_t ic = ok ? i : 0;
#pragma unroll
    for (int j = 0; j < FUSE_DMAX; ++j) {
      const int64_t jj = j < d ? j : d - 1;
      const float zv = a.zin[jj * n + ic], dv = dzsrc[jj * n + ic];
      pz[j] = ok ? zv : 0.5f;
      pd[j] = ok ? dv * dzs : 0.0f;
    }
    const double rv = a.rsave[ic];
    pr = ok ? rv : 0.0;
  };
  // the loss scale: reduced by every wave from the forward's partial rows
  // (first launch of a step; workgroup 0 stores the loss), else read; the
  // rows' loads are in flight while the packs are copied
  LossRows lrows;
  if (a.partials) loss_load(a.partials, a.prows, 0, lrows);
  if (n > 0) fetch(blockIdx.x);
  S* sfw = (S*)flds;
  S* sbw = sfw + L.fw_len;
  float* sb = (float*)(sbw + L.bw_len);
  // the lane's own LDS columns, BS apart: z_j at zc[j], its gradient at
  // zc[d + j], zero at zc[2 d], a sink for unused writes at zc[2 d + 1]
  float* zc = (float*)(flds + fuse_z_offset(L.fw_len, L.bw_len, L.bias_len, es)) + threadIdx.x;
  S* stage = (S*)(flds + fuse_stage_offset(L.fw_len, L.bw_len, L.bias_len, es, d, BS));
  copy16(sfw, fw + L.fw_off, L.fw_len * es);
  copy16(sbw, bw + L.bw_off, L.bw_len * es);
  copy16(sb, bias + L.bias_off, L.bias_len * 4);
  zc[2 * d * BS] = 0.0f;
  // per-lane pointers to the columns of the layer's coordinate sets
  const float* zap[FAB];
  float* dzap[FAB];
#pragma unroll
  for (int e = 0; e < FAB; ++e) {
    const int ai = L.a_idx[e];
    const bool act = e < L.na;
    zap[e] = zc + (act ? ai : 2 * d) * BS;
    dzap[e] = zc + (act ? d + ai : 2 * d + 1) * BS;
  }
  float* zbp[NB];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) zbp[jb] = zc + L.b_idx[jb] * BS;
  double scale;
  if (a.partials) {
    double lv[3];
    loss_finish(a.partials, a.prows, lrows, lv);
    scale = lv[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.loss_out[0] = lv[0];
      a.loss_out[1] = lv[1];
      a.loss_out[2] = lv[2];
    }
  } else {
    scale = a.loss[1];
  }
  __syncthreads();
  const LayerLds<OP> W = layer_lds<OP>(sfw, sb, L, L.fw_off, L.bias_off);
  const frag* w3t = (const frag*)sbw;                       // [2][2 NB][32][2]
  const frag* w2t = (const frag*)(sbw + NB * 2048);         // [2][4][32][2]
  const frag* w1t = (const frag*)(sbw + NB * 2048 + 4096);  // [1][4][32][2]
  S* mystage = stage + (size_t)wave * SR * RS;
  f32x16 acc[OWN];
  float bsum[OWN];
#pragma unroll
  for (int k = 0; k < OWN; ++k) {
    acc[k] = zero16();
    bsum[k] = 0.0f;
  }
  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    // the prefetched inputs into the lane's columns (coordinates j >= d
    // write column d - 1 again, with its own value)
#pragma unroll
    for (int j = 0; j < FUSE_DMAX; ++j) {
      const int jj = j < d ? j : d - 1;
      zc[jj * BS] = pz[j];
      zc[(d + jj) * BS] = pd[j];
    }
    const float dlq = (float)(pr * scale);
    float za[FAB];
#pragma unroll
    for (int e = 0; e < FAB; ++e) za[e] = *zap[e];
    fetch(g + gridDim.x);  // in flight while this group is processed
    // network forward, then bins, dQ and dlogit per transformed dim (the
    // incoming gradient of z_j is its column before this layer's update)
    frag h1b[4], h2b[4], dlb[2 * NB];
    mlp_hidden_fb<OP>(za, W, h1b, h2b);
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      f32x16 q = mlp_logits<OP>(h2b, jb, W);
      softmax32(q);
      float* zj = zbp[jb];
      float* dzj = zj + d * BS;
      int b;
      float al, qb;
      cdf_fwd(q, *zj, b, al, qb);
      const float g_out = *dzj;
      float dq[16];
      float sdot = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int k = drow(v, h);
        dq[v] = g_out * ((k < b) ? 1.0f : ((k == b) ? al : 0.0f)) + ((k == b) ? dlq / qb : 0.0f);
        sdot += q[v] * dq[v];
      }
      sdot += xor32(sdot);
#pragma unroll
      for (int v = 0; v < 16; ++v) q[v] = q[v] * (dq[v] - sdot);  // dlogit
      dlb[2 * jb] = to_b<OP>(q, 0);
      dlb[2 * jb + 1] = to_b<OP>(q, 1);
      *dzj = g_out * (float)FK * qb;
    }
    // stage 1: [dlogit rows 0 .. 32 NB | h2 rows 32 NB .. 32 NB + 64]; dW3, db3
#pragma unroll
    for (int kk = 0; kk < 2 * NB; ++kk) stage_put<OP>(mystage, 32 * (kk >> 1), dlb[kk], kk & 1, s, h);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) stage_put<OP>(mystage, 32 * NB + 32 * (kk >> 1), h2b[kk], kk & 1, s, h);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
      const int tau = wave + WV * k;
      if (tau < T3) fuse_contract<OP, WV, SR>(stage, 0, 32 * NB, tau >> 1, tau & 1, acc[k], bsum[k]);
    }
    __syncthreads();
    // dh2 = W3^T dlogit, masked by relu'; stage 2: [dpre2 rows 0 .. 64 | h1 rows 64 .. 128]
    frag d2b[4];
#pragma unroll
    for (int to = 0; to < 2; ++to) {
      f32x16 ac = zero16();
#pragma unroll
      for (int kk = 0; kk < 2 * NB; ++kk) ac = OP::mma(w3t[((to * 2 * NB + kk) * 32 + s) * 2 + h], dlb[kk], ac);
      d2b[2 * to] = to_b<OP>(ac, 0);
      d2b[2 * to + 1] = to_b<OP>(ac, 1);
      FO::mask(d2b[2 * to], h2b[2 * to]);
      FO::mask(d2b[2 * to + 1], h2b[2 * to + 1]);
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      stage_put<OP>(mystage, 32 * (kk >> 1), d2b[kk], kk & 1, s, h);
      stage_put<OP>(mystage, 64 + 32 * (kk >> 1), h1b[kk], kk & 1, s, h);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
      const int tau = wave + WV * k - T3;
      if (tau >= 0 && tau < 4) fuse_contract<OP, WV, SR>(stage, 0, 64, tau >> 1, tau & 1, acc[k], bsum[k]);
    }
    __syncthreads();
    // dh1 = W2^T dpre2, masked; stage 3: [dpre1 rows 0 .. 64 | zA rows 64 .. 96, rows >= |A| zero]
    frag d1b[4];
#pragma unroll
    for (int to = 0; to < 2; ++to) {
      f32x16 ac = zero16();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) ac = OP::mma(w2t[((to * 4 + kk) * 32 + s) * 2 + h], d2b[kk], ac);
      d1b[2 * to] = to_b<OP>(ac, 0);
      d1b[2 * to + 1] = to_b<OP>(ac, 1);
      FO::mask(d1b[2 * to], h1b[2 * to]);
      FO::mask(d1b[2 * to + 1], h1b[2 * to + 1]);
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) stage_put<OP>(mystage, 32 * (kk >> 1), d1b[kk], kk & 1, s, h);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const float val = (e < FAB && h == 0) ? za[e & (FAB - 1)] : 0.0f;
      mystage[(64 + 16 * h + e) * RS + s] = OP::store(val);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
      const int tau = wave + WV * k - T3 - 4;
      if (tau >= 0 && tau < 2) fuse_contract<OP, WV, SR>(stage, 0, 64, tau, 0, acc[k], bsum[k]);
    }
    __syncthreads();
    // dzA = W1^T dpre1: rows a = 4h + r in registers 0..3
    f32x16 d0 = zero16();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) d0 = OP::mma(w1t[(kk * 32 + s) * 2 + h], d1b[kk], d0);
    float dza[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float mine = d0[r], other = xor32(d0[r]);
      dza[r] = h == 0 ? mine : other;
      dza[4 + r] = h == 0 ? other : mine;
    }
#pragma unroll
    for (int e = 0; e < FAB; ++e) *dzap[e] += dza[e];
    const int64_t i = (g * WV + wave) * 32 + s;
    if (i < n && h == 0) {
      for (int j = 0; j < d; ++j) a.dzin[(int64_t)j * n + i] = zc[(d + j) * BS];
    }
  }
  // the workgroup's partial of the parameter block, each element from its owner
  float* out = gpart + (size_t)blockIdx.x * L.n_par;
  const int na = L.na;
  const int oW1 = 0, ob1 = FH * na, oW2 = ob1 + FH, ob2 = oW2 + FH * FH, oW3 = ob2 + FH, ob3 = oW3 + NB * FK * FH;
  const int i32 = lane & 31;
#pragma unroll
  for (int k = 0; k < OWN; ++k) {
    const int tau = wave + WV * k;
    if (tau >= T) continue;
    int wo, bo, ld, ncol, m, n;
    if (tau < T3) { wo = oW3; bo = ob3; ld = FH; ncol = FH; m = tau >> 1; n = tau & 1; }
    else if (tau < T3 + 4) { wo = oW2; bo = ob2; ld = FH; ncol = FH; m = (tau - T3) >> 1; n = (tau - T3) & 1; }
    else { wo = oW1; bo = ob1; ld = na; ncol = na; m = tau - T3 - 4; n = 0; }
    const int col = 32 * n + i32;
    if (col < ncol) {
#pragma unroll
      for (int v = 0; v < 16; ++v) out[wo + (32 * m + drow(v, h)) * ld + col] = acc[k][v];
    }
    if (n == 0) {
      const float tot = bsum[k] + xor32(bsum[k]);
      if (h == 0) out[bo + 32 * m + i32] = tot;
    }
  }
}

// ---------------------------------------------------------------------------
// Gradient reduction (fixed order over workgroup partials) + Adam.
// ---------------------------------------------------------------------------
constexpr int GSPLIT = 8;  // row groups (waves) of the gradient reduction


struct AdamArgs {
  int64_t n_par;
  int rows;              // workgroup partial rows per layer
  const float* grad_in;  // a full gradient (flow_adam), or null: the step's partial rows
  float* grad_out;       // reduced gradient (nullable)
  float* master;
  float* m;
  float* v;
  const double* loss;    // [3]; ok flag at [2] (nullable = always ok)
  float lr, beta1, beta2, eps;
  int step;              // t >= 1
  int do_adam;
  // with Adam: the positions of each parameter in the forward and backward
  // packs and the bias vector (-1: none), updated with the new weight in
  // place of a full re-pack (null: the caller re-packs)
  const int* fw_dst;
  const int* bw_dst;
  const int* b_dst;
  void* fw;
  void* bw;
  float* bias;
};

// Adam for parameter p with gradient g; with the pack positions, the new
// weight also goes into the packs
template <class OP>
__device__ __forceinline__ void adam_update(const AdamArgs& a, int64_t p, float g) {
  if (a.grad_out) a.grad_out[p] = g;
  if (!a.do_adam) return;
  if (a.loss && a.loss[2] == 0.0) return;  // non-finite loss: leave the weights
  const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * g;
  const float v = a.beta2 * a.v[p] + (1.0f - a.beta2) * g * g;
  a.m[p] = m;
  a.v[p] = v;
  const float mh = m / (1.0f - powf(a.beta1, (float)a.step));
  const float vh = v / (1.0f - powf(a.beta2, (float)a.step));
  const float w = a.master[p] - a.lr * mh / (sqrtf(vh) + a.eps);
  a.master[p] = w;
  if (a.fw_dst) {
    const int kf = a.fw_dst[p], kb = a.bw_dst[p], kc = a.b_dst[p];
    if (kf >= 0) ((typename OP::S*)a.fw)[kf] = OP::store(w);
    if (kb >= 0) ((typename OP::S*)a.bw)[kb] = OP::store(w);
    if (kc >= 0) a.bias[kc] = w;
  }
}

// Adam with a caller's full gradient
template <class OP>
__global__ __launch_bounds__(256) void k_flow_adam(const FlowDesc* __restrict__ Dp, AdamArgs a) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= a.n_par) return;
  adam_update<OP>(a, p, a.grad_in[p]);
}

// The gradient of a training step from the workgroup partial rows, then
// Adam: a workgroup of 64 GSPLIT threads takes 64 parameters; wave w sums
// rows w, w + GSPLIT, ... of its lane's parameter (compensated, in row
// order, eight loads in flight), and the GSPLIT waves' sums are added in
// wave order (a fixed order throughout).
template <class OP>
__global__ __launch_bounds__(64 * GSPLIT) void k_flow_gadam(const FlowDesc* __restrict__ Dp, AdamArgs a,
                                                           const float* __restrict__ gpart) {
  __shared__ float part[GSPLIT][64];
  const FlowDesc& D = *Dp;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  float acc = 0.0f;
  if (p < a.n_par) {
    int l = 0;
    while (l + 1 < D.L && p >= D.l[l + 1].p_off) ++l;
    const int q = (int)(p - D.l[l].p_off);
    const int np = D.l[l].n_par;
    const int rows = a.rows;
    const float* base = gpart + (size_t)D.l[l].p_off * rows;
    float c = 0.0f;
    for (int r0 = w; r0 < rows; r0 += 8 * GSPLIT) {
      float v[8];  // eight rows' loads in flight, then added in row order
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int r = r0 + k * GSPLIT;
        v[k] = r < rows ? base[(size_t)r * np + q] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (r0 + k * GSPLIT < rows) {
          const float y = v[k] - c;
          const float t = acc + y;
          c = (t - acc) - y;
          acc = t;
        }
      }
    }
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w != 0 || p >= a.n_par) return;
  float g = 0.0f;
#pragma unroll
  for (int r = 0; r < GSPLIT; ++r) g += part[r][lane];  // fixed order
  adam_update<OP>(a, p, g);
}

// master FP32 weights -> permuted operand packs (OP::S) and FP32 bias pack
template <class OP>
__global__ __launch_bounds__(256) void k_flow_pack(const float* __restrict__ master, const int* __restrict__ fw_src,
                                                   int fw_total, const int* __restrict__ bw_src, int bw_total,
                                                   const int* __restrict__ b_src, int b_total,
                                                   typename OP::S* __restrict__ fw, typename OP::S* __restrict__ bw,
                                                   float* __restrict__ bias) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < fw_total) {
    const int s = fw_src[k];
    fw[k] = OP::store(s >= 0 ? master[s] : 0.0f);
  }
  if (k < bw_total) {
    const int s = bw_src[k];
    bw[k] = OP::store(s >= 0 ? master[s] : 0.0f);
  }
  if (k < b_total) bias[k] = master[b_src[k]];
}

}  // namespace vgx

using namespace vgx;

struct vgx_flow {
  int device = 0;
  hipStream_t stream = nullptr;
  int dim = 0, L = 0, n_bins = 0, hidden = 0;
  int nbm = 1;            // template bound on |B|
  int64_t n_par = 0;
  FlowDesc D{};
  FlowDesc* d_desc = nullptr;   // device copy read by the kernels
  float* master = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  int f32ops = 0;               // 1: FP32-operand validation kernels (OpF32)
  void* fw = nullptr;           // operand packs, sized for 4-byte elements
  void* bw = nullptr;
  float* bias = nullptr;
  int* fw_src = nullptr;
  int* bw_src = nullptr;
  int* b_src = nullptr;
  int* fw_dst = nullptr;  // inverse of fw_src per parameter (-1: none); null if a parameter
  int* bw_dst = nullptr;  // appears twice in one pack
  int* b_dst = nullptr;
  double* loss = nullptr;       // [3]
  double* partials = nullptr;   // [max grid][4]
  int step = 0;
  // training scratch, grown on demand
  int64_t cap_n = 0;
  float* zsave = nullptr;       // [L][d][n]
  double* rsave = nullptr;      // [n]
  double* lqsave = nullptr;     // [n]
  float* dz[2] = {nullptr, nullptr};  // [d][n]
  void* scr = nullptr;          // operand tiles [tiles][srows][32] of OP::S
  float* gpart = nullptr;       // [n_par * grid_w]
  int grid_w = 0;
  int srows = 0;
  double* pinned = nullptr;
  hipEvent_t ready = nullptr;  // orders other streams after the flow's (flow_order_before)
};

namespace vgx {

FlowView flow_view(const vgx_flow* f) {
  FlowView v{};
  v.desc = f->d_desc;
  v.fw = f->fw;
  v.bias = f->bias;
  v.fw_total = f->D.fw_total;
  v.bias_total = f->D.bias_total;
  v.dim = f->dim;
  v.L = f->L;
  v.nbm = f->nbm;
  v.f32ops = f->f32ops;
  return v;
}

vgx_status flow_order_before(vgx_flow* f, hipStream_t s) {
  if (s == f->stream) return VGX_OK;
  if (!f->ready) VGX_HIP(hipEventCreateWithFlags(&f->ready, hipEventDisableTiming));
  VGX_HIP(hipEventRecord(f->ready, f->stream));
  VGX_HIP(hipStreamWaitEvent(s, f->ready, 0));
  return VGX_OK;
}

}  // namespace vgx

namespace {

int n_bits(int d) {
  int b = 0;
  while ((1 << b) < d) ++b;
  return b < 1 ? 1 : b;
}

vgx_status build_desc(int dim, int L, FlowDesc& D, std::vector<int>& fws, std::vector<int>& bws,
                      std::vector<int>& bs, int64_t& n_par, int& nbm) {
  D = FlowDesc{};
  D.d = dim;
  D.L = L;
  const int nbit = n_bits(dim);
  int p = 0;
  nbm = 1;
  fws.clear();
  bws.clear();
  bs.clear();
  for (int l = 0; l < L; ++l) {
    FlowLayerDesc& Ld = D.l[l];
    const int k = (l / 2) % nbit;
    const int par = (l % 2 == 0) ? 1 : 0;
    Ld.na = Ld.nb = 0;
    for (int j = 0; j < dim; ++j) {
      if (((j >> k) & 1) == par) {
        if (Ld.nb >= FAB) { set_error("flow: |B| > %d", FAB); return VGX_EINVAL; }
        Ld.b_idx[Ld.nb++] = j;
      } else {
        if (Ld.na >= FAB) { set_error("flow: |A| > %d", FAB); return VGX_EINVAL; }
        Ld.a_idx[Ld.na++] = j;
      }
    }
    if (Ld.na == 0 || Ld.nb == 0) { set_error("flow: dimension too small for the masks"); return VGX_EINVAL; }
    const int na = Ld.na, nb = Ld.nb;
    while (nbm < nb) nbm *= 2;
    const int oW1 = p, ob1 = oW1 + FH * na, oW2 = ob1 + FH, ob2 = oW2 + FH * FH, oW3 = ob2 + FH,
              ob3 = oW3 + nb * FK * FH;
    Ld.p_off = p;
    Ld.n_par = FH * na + FH + FH * FH + FH + nb * FK * FH + nb * FK;
    p += Ld.n_par;
    // forward pack
    Ld.fw_off = (int)fws.size();
    for (int t = 0; t < 2; ++t)
      for (int i = 0; i < 32; ++i)
        for (int h = 0; h < 2; ++h)
          for (int e = 0; e < 8; ++e) {
            const int slot = 8 * h + e;
            fws.push_back(slot < na ? oW1 + (32 * t + i) * na + slot : -1);
          }
    for (int t = 0; t < 2; ++t)
      for (int kk = 0; kk < 4; ++kk)
        for (int i = 0; i < 32; ++i)
          for (int h = 0; h < 2; ++h)
            for (int e = 0; e < 8; ++e) {
              const int fin = 16 * kk + 8 * (e >> 2) + 4 * h + (e & 3);
              fws.push_back(oW2 + (32 * t + i) * FH + fin);
            }
    for (int t = 0; t < nb; ++t)
      for (int kk = 0; kk < 4; ++kk)
        for (int i = 0; i < 32; ++i)
          for (int h = 0; h < 2; ++h)
            for (int e = 0; e < 8; ++e) {
              const int fin = 16 * kk + 8 * (e >> 2) + 4 * h + (e & 3);
              fws.push_back(oW3 + (32 * t + i) * FH + fin);
            }
    Ld.fw_len = (int)fws.size() - Ld.fw_off;
    // backward pack: W3^T, W2^T, W1^T
    Ld.bw_off = (int)bws.size();
    for (int t = 0; t < 2; ++t)
      for (int kk = 0; kk < 2 * nb; ++kk)
        for (int i = 0; i < 32; ++i)
          for (int h = 0; h < 2; ++h)
            for (int e = 0; e < 8; ++e) {
              const int o = 16 * kk + 8 * (e >> 2) + 4 * h + (e & 3);
              bws.push_back(oW3 + o * FH + 32 * t + i);
            }
    for (int t = 0; t < 2; ++t)
      for (int kk = 0; kk < 4; ++kk)
        for (int i = 0; i < 32; ++i)
          for (int h = 0; h < 2; ++h)
            for (int e = 0; e < 8; ++e) {
              const int f = 16 * kk + 8 * (e >> 2) + 4 * h + (e & 3);
              bws.push_back(oW2 + f * FH + 32 * t + i);
            }
    for (int kk = 0; kk < 4; ++kk)
      for (int i = 0; i < 32; ++i)
        for (int h = 0; h < 2; ++h)
          for (int e = 0; e < 8; ++e) {
            const int f = 16 * kk + 8 * (e >> 2) + 4 * h + (e & 3);
            bws.push_back(i < na ? oW1 + f * na + i : -1);
          }
    Ld.bw_len = (int)bws.size() - Ld.bw_off;
    // biases
    Ld.bias_off = (int)bs.size();
    for (int f = 0; f < FH; ++f) bs.push_back(ob1 + f);
    for (int f = 0; f < FH; ++f) bs.push_back(ob2 + f);
    for (int o = 0; o < nb * FK; ++o) bs.push_back(ob3 + o);
    Ld.bias_len = (int)bs.size() - Ld.bias_off;
  }
  D.fw_total = (int)fws.size();
  D.bw_total = (int)bws.size();
  D.bias_total = (int)bs.size();
  n_par = p;
  return VGX_OK;
}

int op_es(const vgx_flow* f) { return f->f32ops ? 4 : 2; }

size_t bwd_lds(const vgx_flow* f, int l) {
  const FlowLayerDesc& Ld = f->D.l[l];
  return bwd_z_offset(Ld.fw_len, Ld.bw_len, Ld.bias_len, op_es(f)) + sizeof(float) * 3 * (size_t)f->dim * FBLOCK;
}

template <class OP>
size_t fuse_lds_wv(const vgx_flow* f, int l, int wv) {
  const FlowLayerDesc& Ld = f->D.l[l];
  const int es = (int)sizeof(typename OP::S);
  return fuse_stage_offset(Ld.fw_len, Ld.bw_len, Ld.bias_len, es, f->dim, 64 * wv) +
         (size_t)wv * fuse_stage_rows(Ld.nb) * fuse_rs<OP>() * es;
}

// waves of the fused workgroup of layer l: eight (two per SIMD, so that one
// wave's waits overlap the other's work) for BF16 operands and |B| <= 2
// where their stages fit the LDS, else four
template <class OP>
int fuse_waves(const vgx_flow* f, int l) {
  return (sizeof(typename OP::S) == 2 && f->D.l[l].nb <= 2 && fuse_lds_wv<OP>(f, l, 8) <= 160 * 1024) ? 8 : 4;
}

template <class OP>
size_t fuse_lds_op(const vgx_flow* f, int l) { return fuse_lds_wv<OP>(f, l, fuse_waves<OP>(f, l)); }

size_t fuse_lds(const vgx_flow* f, int l) { return f->f32ops ? fuse_lds_op<OpF32>(f, l) : fuse_lds_op<OpBF16>(f, l); }

// the fused kernel of a layer with |B| = nb and wv waves
template <class OP>
const void* fuse_kernel(int nb, int wv) {
  if (wv == 8) {
    if constexpr (sizeof(typename OP::S) == 2) {
      switch (nb) {
        case 1: return (const void*)k_flow_bwdw<1, 8, OP>;
        case 2: return (const void*)k_flow_bwdw<2, 8, OP>;
        default: return nullptr;
      }
    }
    return nullptr;
  }
  switch (nb) {
    case 1: return (const void*)k_flow_bwdw<1, 4, OP>;
    case 2: return (const void*)k_flow_bwdw<2, 4, OP>;
    case 3: return (const void*)k_flow_bwdw<3, 4, OP>;
    case 4: return (const void*)k_flow_bwdw<4, 4, OP>;
    default: return nullptr;
  }
}

// allow every fused kernel the whole LDS of a CU (a launch still asks only
// for what its layer needs), once per process
template <class OP>
vgx_status fuse_allow_lds() {
  static bool done = false;
  if (done) return VGX_OK;
  for (int nb = 1; nb <= 4; ++nb)
    for (int wv = 4; wv <= 8; wv += 4)
      if (const void* k = fuse_kernel<OP>(nb, wv))
        VGX_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  done = true;
  return VGX_OK;
}

// the backward of layers with |B| <= 4 runs fused with its weight gradients
bool fused_backward(const vgx_flow* f) { return f->nbm <= 4; }

size_t fwd_lds_es(const vgx_flow* f, int es) {
  return fwd_z_offset(f->D.fw_total, f->D.bias_total, es) + sizeof(float) * (size_t)f->dim * FWD_BLOCK;
}

size_t fwd_lds(const vgx_flow* f) { return fwd_lds_es(f, op_es(f)); }

vgx_status pack(vgx_flow* f) {
  const int tot = f->D.fw_total > f->D.bw_total ? f->D.fw_total : f->D.bw_total;
  if (f->f32ops)
    hipLaunchKernelGGL(k_flow_pack<OpF32>, dim3((tot + 255) / 256), dim3(256), 0, f->stream, f->master, f->fw_src,
                       f->D.fw_total, f->bw_src, f->D.bw_total, f->b_src, f->D.bias_total, (float*)f->fw,
                       (float*)f->bw, f->bias);
  else
    hipLaunchKernelGGL(k_flow_pack<OpBF16>, dim3((tot + 255) / 256), dim3(256), 0, f->stream, f->master, f->fw_src,
                       f->D.fw_total, f->bw_src, f->D.bw_total, f->b_src, f->D.bias_total, (unsigned short*)f->fw,
                       (unsigned short*)f->bw, f->bias);
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

// Allow the dynamic LDS the kernels of this flow need (beyond 64 KB), once.
template <int NB, class OP>
vgx_status set_lds_limits(size_t fwd, size_t bwd, size_t wgr, size_t fus) {
  // never lower a limit another live flow may rely on
  static size_t cur_f = 0, cur_b = 0, cur_w = 0, cur_u = 0;
  fwd = fwd > cur_f ? fwd : cur_f;
  bwd = bwd > cur_b ? bwd : cur_b;
  wgr = wgr > cur_w ? wgr : cur_w;
  fus = fus > cur_u ? fus : cur_u;
  cur_f = fwd;
  cur_b = bwd;
  cur_w = wgr;
  cur_u = fus;
  if (fus > 0) VGX_TRY(fuse_allow_lds<OP>());
  VGX_HIP(hipFuncSetAttribute((const void*)k_flow_fwd<NB, 0, OP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd));
  VGX_HIP(hipFuncSetAttribute((const void*)k_flow_fwd<NB, 1, OP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd));
  VGX_HIP(hipFuncSetAttribute((const void*)k_flow_fwd<NB, 2, OP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd));
  if constexpr (NB > 4) {
    VGX_HIP(hipFuncSetAttribute((const void*)k_flow_bwd<NB, OP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwd));
    VGX_HIP(hipFuncSetAttribute((const void*)k_flow_wgrad<NB, OP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)wgr));
  }
  return VGX_OK;
}

template <class OP>
vgx_status set_lds_limits_nb(int nbm, size_t fwd, size_t bwd, size_t wgr, size_t fus) {
  switch (nbm) {
    case 1: return set_lds_limits<1, OP>(fwd, bwd, wgr, fus);
    case 2: return set_lds_limits<2, OP>(fwd, bwd, wgr, fus);
    case 4: return set_lds_limits<4, OP>(fwd, bwd, wgr, fus);
    default: return set_lds_limits<8, OP>(fwd, bwd, wgr, fus);
  }
}

vgx_status init_lds_limits(const vgx_flow* f) {
  size_t fwd = fwd_lds(f), bwd = 0, wgr = 0, fus = 0;
  for (int l = 0; l < f->L; ++l) {
    const FlowLayerDesc& Ld = f->D.l[l];
    const size_t b = bwd_lds(f, l);
    bwd = b > bwd ? b : bwd;
    wgr = (size_t)Ld.n_par * 4 > wgr ? (size_t)Ld.n_par * 4 : wgr;
    if (fused_backward(f)) fus = std::max(fus, fuse_lds(f, l));
  }
  return f->f32ops ? set_lds_limits_nb<OpF32>(f->nbm, fwd, bwd, wgr, fus)
                   : set_lds_limits_nb<OpBF16>(f->nbm, fwd, bwd, wgr, fus);
}

// forward grid: tile pairs go round-robin over the workgroups (wave w of
// workgroup b takes pairs w gridDim + b, ...), so a batch of fewer than
// FWD_BLOCK / 64 pairs per CU still spreads over every CU
int fwd_grid(const vgx_flow* f, int64_t n, int per_cu = 2) {
  const int64_t tiles = (n + 63) / 64;  // the forward kernels take 64-sample tile pairs
  int64_t g = tiles;
  const int64_t cap = (int64_t)device_cus() * per_cu;
  if (g > cap) g = cap;
  return (int)(g < 1 ? 1 : g);
}

template <int MODE, class OP>
vgx_status launch_fwd_op(vgx_flow* f, int grid, const FwdArgs& a, hipStream_t st) {
  const size_t lds = fwd_lds(f);
  const typename OP::S* fw = (const typename OP::S*)f->fw;
#define L_(NB)                                                                                                  \
  case NB:                                                                                                      \
    hipLaunchKernelGGL((k_flow_fwd<NB, MODE, OP>), dim3(grid), dim3(FWD_BLOCK), lds, st, f->d_desc, a, fw, f->bias); \
    break;
  switch (f->nbm) { L_(1) L_(2) L_(4) L_(8) default: set_error("flow: bad |B| bound"); return VGX_EINVAL; }
#undef L_
  VGX_HIP(hipGetLastError());
  return VGX_OK;
}

template <int MODE>
vgx_status launch_fwd(vgx_flow* f, int grid, const FwdArgs& a, hipStream_t st) {
  return f->f32ops ? launch_fwd_op<MODE, OpF32>(f, grid, a, st) : launch_fwd_op<MODE, OpBF16>(f, grid, a, st);
}

vgx_status ensure_train(vgx_flow* f, int64_t n) {
  if (n <= f->cap_n) return VGX_OK;
  hipFree(f->zsave); hipFree(f->rsave); hipFree(f->lqsave); hipFree(f->dz[0]); hipFree(f->dz[1]); hipFree(f->scr);
  hipFree(f->gpart);
  f->zsave = nullptr; f->rsave = nullptr; f->lqsave = nullptr; f->dz[0] = f->dz[1] = nullptr; f->scr = nullptr;
  f->gpart = nullptr;
  f->cap_n = 0;
  const int64_t tiles = (n + 31) / 32;
  const size_t es = (size_t)op_es(f);
  f->srows = 32 + 4 * FH + FK * f->nbm;
  f->grid_w = device_cus();
  VGX_TRY(dev_alloc((void**)&f->zsave, sizeof(float) * (size_t)f->L * f->dim * n));
  VGX_TRY(dev_alloc((void**)&f->rsave, sizeof(double) * (size_t)n));
  VGX_TRY(dev_alloc((void**)&f->lqsave, sizeof(double) * (size_t)n));
  VGX_TRY(dev_alloc((void**)&f->dz[0], sizeof(float) * (size_t)f->dim * n));
  VGX_TRY(dev_alloc((void**)&f->dz[1], sizeof(float) * (size_t)f->dim * n));
  if (!fused_backward(f)) VGX_TRY(dev_alloc((void**)&f->scr, es * (size_t)tiles * f->srows * 32));
  VGX_TRY(dev_alloc((void**)&f->gpart, sizeof(float) * (size_t)f->n_par * f->grid_w));
  // rows 16..31 of the zA block are never written and must read as zero
  if (f->scr) VGX_HIP(hipMemsetAsync(f->scr, 0, es * (size_t)tiles * f->srows * 32, f->stream));
  f->cap_n = n;
  return VGX_OK;
}

// forward (training) + loss + per-layer backward + weight gradients; leaves
// per-workgroup partials in gpart and the loss on the device.
vgx_status loss_grad_enqueue(vgx_flow* f, int64_t n, const double* y, const double* g) {
  VGX_TRY(ensure_train(f, n));
  // training kernels stage a layer's weights per workgroup: one per CU
  const int grid = fwd_grid(f, n, 1);
  FwdArgs a{};
  a.n = n;
  a.yin = y;
  a.g = g;
  a.out = nullptr;
  a.logq = f->lqsave;
  a.zsave = f->zsave;
  a.rsave = f->rsave;
  a.partials = f->partials;
  VGX_TRY(launch_fwd<1>(f, grid, a, f->stream));
  // the fused backward of the last layer reduces the loss itself
  if (!fused_backward(f)) {
    hipLaunchKernelGGL(k_flow_loss, dim3(1), dim3(64), 0, f->stream, f->partials, grid, f->loss);
    VGX_HIP(hipGetLastError());
  }
  const int wgrid = f->grid_w;
  // backward: two resident workgroups per CU (the layer's packs in LDS)
  const int64_t btiles = (n + 31) / 32;
  const int bgrid = (int)std::min<int64_t>(std::max<int64_t>((btiles + 3) / 4, 1), 2 * (int64_t)device_cus());
  int cur = 0;
  for (int l = f->L - 1; l >= 0; --l) {
    const FlowLayerDesc& Ld = f->D.l[l];
    BwdArgs b{};
    b.n = n;
    b.layer = l;
    b.zin = f->zsave + (size_t)l * f->dim * n;
    b.dzout = (l == f->L - 1) ? nullptr : f->dz[cur];
    b.dzin = f->dz[cur ^ 1];
    b.rsave = f->rsave;
    b.loss = f->loss;
    b.scr = f->scr;
    b.srows = f->srows;
    b.partials = l == f->L - 1 ? f->partials : nullptr;
    b.prows = grid;
    b.loss_out = f->loss;
    const size_t wl = (size_t)Ld.n_par * 4;
    float* gp = f->gpart + (size_t)Ld.p_off * wgrid;
    if (fused_backward(f)) {
      const size_t lds = fuse_lds(f, l);
      const int wv = f->f32ops ? fuse_waves<OpF32>(f, l) : fuse_waves<OpBF16>(f, l);
#define F_(NB, WV, OP)                                                                                    \
  hipLaunchKernelGGL((k_flow_bwdw<NB, WV, OP>), dim3(wgrid), dim3(64 * WV), lds, f->stream, f->d_desc, b, \
                     (const OP::S*)f->fw, (const OP::S*)f->bw, f->bias, gp)
      const int key = 10 * Ld.nb + wv;
      if (f->f32ops) {
        switch (Ld.nb) {
          case 1: F_(1, 4, OpF32); break;
          case 2: F_(2, 4, OpF32); break;
          case 3: F_(3, 4, OpF32); break;
          case 4: F_(4, 4, OpF32); break;
          default: return VGX_EINVAL;
        }
      } else {
        switch (key) {
          case 14: F_(1, 4, OpBF16); break;
          case 18: F_(1, 8, OpBF16); break;
          case 24: F_(2, 4, OpBF16); break;
          case 28: F_(2, 8, OpBF16); break;
          case 34: F_(3, 4, OpBF16); break;
          case 44: F_(4, 4, OpBF16); break;
          default: return VGX_EINVAL;
        }
      }
#undef F_
      VGX_HIP(hipGetLastError());
      cur ^= 1;
      continue;
    }
    const size_t lds = bwd_lds(f, l);
#define B_(NB, OP)                                                                                        \
  case NB:                                                                                                \
    hipLaunchKernelGGL((k_flow_bwd<NB, OP>), dim3(bgrid), dim3(FBLOCK), lds, f->stream, f->d_desc, b,     \
                       (const OP::S*)f->fw, (const OP::S*)f->bw, f->bias);                                \
    break;
    // |B| up to 8: backward and weight gradients as two kernels
    if (f->f32ops) {
      switch (f->nbm) { B_(8, OpF32) default: return VGX_EINVAL; }
    } else {
      switch (f->nbm) { B_(8, OpBF16) default: return VGX_EINVAL; }
    }
#undef B_
    VGX_HIP(hipGetLastError());
    WgradArgs w{};
    w.n = n;
    w.layer = l;
    w.scr = f->scr;
    w.srows = f->srows;
    w.gpart = gp;
#define W_(NB, OP)                                                                                    \
  case NB:                                                                                            \
    hipLaunchKernelGGL((k_flow_wgrad<NB, OP>), dim3(wgrid), dim3(FBLOCK), wl, f->stream, f->d_desc, w); \
    break;
    if (f->f32ops) {
      switch (f->nbm) { W_(8, OpF32) default: return VGX_EINVAL; }
    } else {
      switch (f->nbm) { W_(8, OpBF16) default: return VGX_EINVAL; }
    }
#undef W_
    VGX_HIP(hipGetLastError());
    cur ^= 1;
  }
  return VGX_OK;
}

vgx_status reduce_adam(vgx_flow* f, const float* grad_in, float* grad_out, float lr, bool adam, const double* loss) {
  AdamArgs a{};
  a.n_par = f->n_par;
  a.rows = f->grid_w;
  a.grad_in = grad_in;
  a.grad_out = grad_out;
  a.master = f->master;
  a.m = f->m;
  a.v = f->v;
  a.loss = loss;
  a.lr = lr;
  a.beta1 = 0.9f;
  a.beta2 = 0.999f;
  a.eps = 1e-8f;
  a.do_adam = adam ? 1 : 0;
  if (adam) a.step = ++f->step;
  if (adam && f->fw_dst) {
    a.fw_dst = f->fw_dst;
    a.bw_dst = f->bw_dst;
    a.b_dst = f->b_dst;
    a.fw = f->fw;
    a.bw = f->bw;
    a.bias = f->bias;
  }
  if (grad_in) {
    const dim3 grid((unsigned)((f->n_par + 255) / 256));
    if (f->f32ops)
      hipLaunchKernelGGL(k_flow_adam<OpF32>, grid, dim3(256), 0, f->stream, f->d_desc, a);
    else
      hipLaunchKernelGGL(k_flow_adam<OpBF16>, grid, dim3(256), 0, f->stream, f->d_desc, a);
  } else {
    // the workgroup partials of the training step, reduced and applied at once
    const dim3 grid((unsigned)((f->n_par + 63) / 64));
    if (f->f32ops)
      hipLaunchKernelGGL(k_flow_gadam<OpF32>, grid, dim3(64 * GSPLIT), 0, f->stream, f->d_desc, a, f->gpart);
    else
      hipLaunchKernelGGL(k_flow_gadam<OpBF16>, grid, dim3(64 * GSPLIT), 0, f->stream, f->d_desc, a, f->gpart);
  }
  VGX_HIP(hipGetLastError());
  if (adam && !f->fw_dst) VGX_TRY(pack(f));
  return VGX_OK;
}

}  // namespace

extern "C" int64_t flow_num_params(int32_t dim, int32_t n_layers, int32_t n_bins, int32_t hidden) {
  if (dim < 2 || dim > VGX_MAX_DIM || n_layers < 1 || n_layers > FL_MAX || n_bins != FK || hidden != FH) return -1;
  FlowDesc D;
  std::vector<int> a, b, c;
  int64_t np = 0;
  int nbm = 0;
  if (build_desc(dim, n_layers, D, a, b, c, np, nbm) != VGX_OK) return -1;
  return np;
}

extern "C" vgx_status flow_shape(const vgx_flow* f, int32_t* dim, int64_t* n_params) {
  VGX_CHECK(f, "flow_shape: null flow");
  if (dim) *dim = f->dim;
  if (n_params) *n_params = f->n_par;
  return VGX_OK;
}

extern "C" vgx_status flow_param_layout(int32_t dim, int32_t n_layers, int32_t n_bins, int32_t hidden,
                                       int32_t* kind, int32_t* fan_in, int64_t* size, int32_t cap, int32_t* n_seg) {
  VGX_CHECK(n_seg, "flow_param_layout: null n_seg");
  VGX_CHECK(dim >= 2 && dim <= VGX_MAX_DIM && n_layers >= 1 && n_layers <= FL_MAX && n_bins == FK && hidden == FH,
            "flow_param_layout: unsupported shape");
  FlowDesc D;
  std::vector<int> a, b, c;
  int64_t np = 0;
  int nbm = 0;
  VGX_TRY(build_desc(dim, n_layers, D, a, b, c, np, nbm));
  *n_seg = 6 * n_layers;
  int k = 0;
  for (int l = 0; l < n_layers; ++l) {
    const int na = D.l[l].na, nb = D.l[l].nb;
    const int32_t kd[6] = {0, 1, 0, 1, 2, 2};
    const int32_t fi[6] = {na, na, FH, FH, FH, FH};
    const int64_t sz[6] = {(int64_t)FH * na, FH, (int64_t)FH * FH, FH, (int64_t)nb * FK * FH, (int64_t)nb * FK};
    for (int q = 0; q < 6; ++q, ++k) {
      if (k >= cap) continue;
      if (kind) kind[k] = kd[q];
      if (fan_in) fan_in[k] = fi[q];
      if (size) size[k] = sz[q];
    }
  }
  return VGX_OK;
}

extern "C" vgx_status flow_create(int32_t dim, int32_t n_layers, int32_t n_bins, int32_t hidden, const float* params,
                                  int64_t n_params, void* stream, vgx_flow** out) {
  VGX_CHECK(out, "flow_create: null out");
  *out = nullptr;
  VGX_CHECK(dim >= 2 && dim <= VGX_MAX_DIM, "flow_create: dim %d out of 2..%d", dim, VGX_MAX_DIM);
  VGX_CHECK(n_layers >= 1 && n_layers <= FL_MAX, "flow_create: n_layers out of 1..%d", FL_MAX);
  VGX_CHECK(n_bins == FK && hidden == FH, "flow_create: supported n_bins = %d, hidden = %d", FK, FH);
  VGX_CHECK(params, "flow_create: null params");
  vgx_flow* f = new vgx_flow();
  hipGetDevice(&f->device);
  f->stream = (hipStream_t)stream;
  f->dim = dim;
  f->L = n_layers;
  f->n_bins = n_bins;
  f->hidden = hidden;
  std::vector<int> fws, bws, bs;
  vgx_status s = build_desc(dim, n_layers, f->D, fws, bws, bs, f->n_par, f->nbm);
  if (s != VGX_OK) { delete f; return s; }
  if (n_params != f->n_par) {
    delete f;
    set_error("flow_create: expected %lld parameters, got %lld", (long long)f->n_par, (long long)n_params);
    return VGX_EINVAL;
  }
  size_t need = fwd_lds(f);
  if (fused_backward(f))
    for (int l = 0; l < f->L; ++l) need = std::max(need, fuse_lds(f, l));
  if (need > 160 * 1024) {
    delete f;
    set_error("flow_create: packed weights exceed LDS");
    return VGX_EINVAL;
  }
  // each parameter's position in the packs: Adam writes the new weight
  // there directly (only if no parameter appears twice in one pack)
  std::vector<int> fwd(f->n_par, -1), bwd(f->n_par, -1), bd(f->n_par, -1);
  bool inv_ok = true;
  auto invert = [&](const std::vector<int>& src, std::vector<int>& dst) {
    for (size_t k = 0; k < src.size(); ++k) {
      const int q = src[k];
      if (q < 0) continue;
      if (q >= f->n_par || dst[q] >= 0) inv_ok = false;
      else dst[q] = (int)k;
    }
  };
  invert(fws, fwd);
  invert(bws, bwd);
  invert(bs, bd);
  do {
    if ((s = dev_alloc((void**)&f->master, sizeof(float) * f->n_par)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->m, sizeof(float) * f->n_par)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->v, sizeof(float) * f->n_par)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->grad, sizeof(float) * f->n_par)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->fw, 4 * (size_t)f->D.fw_total)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->bw, 4 * (size_t)f->D.bw_total)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->bias, 4 * (size_t)f->D.bias_total)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->fw_src, 4 * fws.size())) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->bw_src, 4 * bws.size())) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->b_src, 4 * bs.size())) != VGX_OK) break;
    if (inv_ok) {
      if ((s = dev_alloc((void**)&f->fw_dst, 4 * (size_t)f->n_par)) != VGX_OK) break;
      if ((s = dev_alloc((void**)&f->bw_dst, 4 * (size_t)f->n_par)) != VGX_OK) break;
      if ((s = dev_alloc((void**)&f->b_dst, 4 * (size_t)f->n_par)) != VGX_OK) break;
    }
    if ((s = dev_alloc((void**)&f->loss, sizeof(double) * 4)) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->d_desc, sizeof(FlowDesc))) != VGX_OK) break;
    if ((s = dev_alloc((void**)&f->partials, sizeof(double) * 4 * (size_t)device_cus() * 2)) != VGX_OK) break;
    if ((s = host_alloc((void**)&f->pinned, sizeof(double) * 4)) != VGX_OK) break;
  } while (0);
  if (s != VGX_OK) { flow_destroy(f); return s; }
  hipError_t e = hipMemcpyAsync(f->master, params, sizeof(float) * f->n_par, hipMemcpyHostToDevice, f->stream);
  if (e == hipSuccess) e = hipMemsetAsync(f->m, 0, sizeof(float) * f->n_par, f->stream);
  if (e == hipSuccess) e = hipMemsetAsync(f->v, 0, sizeof(float) * f->n_par, f->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f->fw_src, fws.data(), 4 * fws.size(), hipMemcpyHostToDevice, f->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f->bw_src, bws.data(), 4 * bws.size(), hipMemcpyHostToDevice, f->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f->b_src, bs.data(), 4 * bs.size(), hipMemcpyHostToDevice, f->stream);
  if (inv_ok) {
    if (e == hipSuccess) e = hipMemcpyAsync(f->fw_dst, fwd.data(), 4 * fwd.size(), hipMemcpyHostToDevice, f->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f->bw_dst, bwd.data(), 4 * bwd.size(), hipMemcpyHostToDevice, f->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f->b_dst, bd.data(), 4 * bd.size(), hipMemcpyHostToDevice, f->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(f->d_desc, &f->D, sizeof(FlowDesc), hipMemcpyHostToDevice, f->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);  // host vectors die at return
  if (e != hipSuccess) { s = hip_fail(e, "flow_create copies", __FILE__, __LINE__); flow_destroy(f); return s; }
  s = init_lds_limits(f);
  if (s == VGX_OK) s = pack(f);
  if (s == VGX_OK) {
    e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) s = hip_fail(e, "flow_create pack", __FILE__, __LINE__);
  }
  if (s != VGX_OK) { flow_destroy(f); return s; }
  *out = f;
  return VGX_OK;
}

extern "C" vgx_status flow_set_operands(vgx_flow* f, int32_t operands) {
  VGX_CHECK(f, "flow_set_operands: null flow");
  VGX_CHECK(operands == VGX_OPERANDS_BF16 || operands == VGX_OPERANDS_F32, "flow_set_operands: unknown mode %d",
            operands);
  const int want = operands == VGX_OPERANDS_F32 ? 1 : 0;
  if (want == f->f32ops) return VGX_OK;
  size_t need = fwd_lds_es(f, want ? 4 : 2);
  if (fused_backward(f))
    for (int l = 0; l < f->L; ++l)
      need = std::max(need, want ? fuse_lds_op<OpF32>(f, l) : fuse_lds_op<OpBF16>(f, l));
  if (need > 160 * 1024) {
    set_error("flow_set_operands: the FP32 weight packs of a %d-dimensional flow exceed the LDS", f->dim);
    return VGX_EINVAL;
  }
  VGX_HIP(hipStreamSynchronize(f->stream));
  // the training tiles change element size: reallocated on the next use
  hipFree(f->zsave); hipFree(f->rsave); hipFree(f->lqsave); hipFree(f->dz[0]); hipFree(f->dz[1]); hipFree(f->scr);
  hipFree(f->gpart);
  f->zsave = nullptr; f->rsave = nullptr; f->lqsave = nullptr; f->dz[0] = f->dz[1] = nullptr; f->scr = nullptr;
  f->gpart = nullptr;
  f->cap_n = 0;
  f->f32ops = want;
  VGX_TRY(init_lds_limits(f));
  VGX_TRY(pack(f));
  VGX_HIP(hipStreamSynchronize(f->stream));
  return VGX_OK;
}

extern "C" vgx_status flow_sample(vgx_flow* f, int64_t n, uint64_t seed, uint32_t stream_id, int32_t iteration,
                                  double* y, double* logq, void* stream) {
  VGX_CHECK(f, "flow_sample: null flow");
  VGX_CHECK(n >= 0 && stream_id < (1u << 23), "flow_sample: bad n or stream_id");
  if (n == 0) return VGX_OK;
  VGX_CHECK(y && logq, "flow_sample: null output");
  FwdArgs a{};
  a.n = n;
  a.out = y;
  a.logq = logq;
  a.it = (uint32_t)iteration;
  a.sid = stream_id | (1u << 23);
  a.k0 = (uint32_t)seed;
  a.k1 = (uint32_t)(seed >> 32);
  return launch_fwd<2>(f, fwd_grid(f, n), a, (hipStream_t)stream);
}

extern "C" vgx_status flow_density(vgx_flow* f, int64_t n, const double* y, double* u, double* logq, void* stream) {
  VGX_CHECK(f, "flow_density: null flow");
  VGX_CHECK(n >= 0, "flow_density: n < 0");
  if (n == 0) return VGX_OK;
  VGX_CHECK(y && logq, "flow_density: null pointer");
  FwdArgs a{};
  a.n = n;
  a.yin = y;
  a.out = u;
  a.logq = logq;
  return launch_fwd<0>(f, fwd_grid(f, n), a, (hipStream_t)stream);
}

extern "C" vgx_status flow_loss_grad(vgx_flow* f, int64_t n, const double* y, const double* g, double* loss_host,
                                     float* grad_host) {
  VGX_CHECK(f, "flow_loss_grad: null flow");
  VGX_CHECK(n >= 2 && y && g, "flow_loss_grad: need n >= 2 and data");
  VGX_TRY(loss_grad_enqueue(f, n, y, g));
  VGX_TRY(reduce_adam(f, nullptr, f->grad, 0.0f, false, nullptr));
  VGX_HIP(hipMemcpyAsync(f->pinned, f->loss, sizeof(double) * 3, hipMemcpyDeviceToHost, f->stream));
  if (grad_host) VGX_HIP(hipMemcpyAsync(grad_host, f->grad, sizeof(float) * f->n_par, hipMemcpyDeviceToHost, f->stream));
  VGX_HIP(hipStreamSynchronize(f->stream));
  if (loss_host) *loss_host = f->pinned[0];
  return VGX_OK;
}

extern "C" vgx_status flow_train_step(vgx_flow* f, int64_t n, const double* y, const double* g, float lr,
                                      double* loss_host) {
  VGX_CHECK(f, "flow_train_step: null flow");
  VGX_CHECK(n >= 2 && y && g, "flow_train_step: need n >= 2 and data");
  VGX_CHECK(lr >= 0.0f, "flow_train_step: lr < 0");
  VGX_TRY(loss_grad_enqueue(f, n, y, g));
  VGX_TRY(reduce_adam(f, nullptr, f->grad, lr, true, f->loss));
  if (!loss_host) return VGX_OK;
  VGX_HIP(hipMemcpyAsync(f->pinned, f->loss, sizeof(double) * 3, hipMemcpyDeviceToHost, f->stream));
  VGX_HIP(hipStreamSynchronize(f->stream));
  *loss_host = f->pinned[0];
  if (f->pinned[2] == 0.0) {
    --f->step;  // the update was skipped on the device
    set_error("flow_train_step: non-finite loss, weights unchanged");
    return VGX_EFALLBACK;
  }
  return VGX_OK;
}

extern "C" vgx_status flow_adam(vgx_flow* f, const float* grad, float lr) {
  VGX_CHECK(f && grad, "flow_adam: null argument");
  return reduce_adam(f, grad, nullptr, lr, true, nullptr);
}

extern "C" vgx_status flow_get_params(vgx_flow* f, float* params, int64_t cap, int64_t* n) {
  VGX_CHECK(f && n, "flow_get_params: null argument");
  *n = f->n_par;
  if (!params || cap < f->n_par) return VGX_OK;
  VGX_HIP(hipMemcpyAsync(params, f->master, sizeof(float) * f->n_par, hipMemcpyDeviceToHost, f->stream));
  VGX_HIP(hipStreamSynchronize(f->stream));
  return VGX_OK;
}

extern "C" vgx_status flow_set_params(vgx_flow* f, const float* params, int64_t n) {
  VGX_CHECK(f && params, "flow_set_params: null argument");
  VGX_CHECK(n == f->n_par, "flow_set_params: expected %lld parameters", (long long)f->n_par);
  VGX_HIP(hipMemcpyAsync(f->master, params, sizeof(float) * n, hipMemcpyHostToDevice, f->stream));
  VGX_TRY(pack(f));
  VGX_HIP(hipStreamSynchronize(f->stream));
  return VGX_OK;
}

extern "C" void flow_destroy(vgx_flow* f) {
  if (!f) return;
  if (f->stream) hipStreamSynchronize(f->stream);
  hipFree(f->master); hipFree(f->m); hipFree(f->v); hipFree(f->grad);
  hipFree(f->fw); hipFree(f->bw); hipFree(f->bias);
  hipFree(f->fw_src); hipFree(f->bw_src); hipFree(f->b_src);
  hipFree(f->fw_dst); hipFree(f->bw_dst); hipFree(f->b_dst);
  hipFree(f->loss); hipFree(f->partials); hipFree(f->d_desc);
  hipFree(f->zsave); hipFree(f->rsave); hipFree(f->lqsave); hipFree(f->dz[0]); hipFree(f->dz[1]); hipFree(f->scr); hipFree(f->gpart);
  if (f->ready) hipEventDestroy(f->ready);
  if (f->pinned) hipHostFree(f->pinned);
  delete f;
}
