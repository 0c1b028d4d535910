// Spectrum surrogate: 2 -> 256 -> 256 -> 256 -> 64 perceptron with GELU,
// trained and evaluated on the matrix cores.
//
// Every product is C[M][N] = A[M][K] Bt[N][K]^T with BF16 operands stored
// K-contiguous and FP32 accumulation (v_mfma_f32_16x16x32_bf16):
//   forward          a_l   = h_{l-1} W_l^T            (A = h_{l-1},  Bt = W_l)
//   input gradient   dh    = da_l W_l                 (A = da_l,     Bt = W_l^T)
//   weight gradient  gW_l  = da_l^T h_{l-1}           (A = da_l^T,   Bt = h_{l-1}^T)
// A training step is three kernels.  The first takes 16 batch rows per block
// through the forward pass, the loss and the input-gradient chain with the
// activations in LDS (all of that is local to a row), and writes BF16
// transposed copies of h_l and da_l.  The second computes the three weight
// gradients in one launch, split over the batch (KSPLIT rows per split).  The
// third sums every partial (splits, bias columns, loss) in a fixed order and
// applies Adam, so a training step is deterministic.
//
// Operand layout of one 16x16x32 product on a 64-lane wave (verified on the
// device): lane l holds A[l%16][8(l/16) .. 8(l/16)+7] and
// Bt[l%16][8(l/16) .. 8(l/16)+7] (8 BF16 each) and receives
// C[4(l/16) + e][l%16], e = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "../../include/surrogate.h"

using namespace cl;

struct surrogate_t;

namespace {

constexpr int NIN = SURR_N_IN, WID = SURR_WIDTH, NOUT = SURR_N_OUT, NPAR = SURR_NPARAMS;
constexpr int NFQ0 = SURR_N_FREQ0, NFQ1 = SURR_N_FREQ1, NFEAT = SURR_N_FEAT;
static_assert(NFEAT == NIN + 2 * (NFQ0 + NFQ1), "feature count");
// offsets of the tensors in the flat parameter vector
constexpr int OW1 = 0, OB1 = OW1 + WID * NFEAT, OW2 = OB1 + WID, OB2 = OW2 + WID * WID, OW3 = OB2 + WID,
              OB3 = OW3 + WID * WID, OW4 = OB3 + WID, OB4 = OW4 + NOUT * WID;
static_assert(OB4 + NOUT == NPAR, "parameter count");

constexpr int KSPLIT = 256;      // batch rows per split of a weight-gradient product
constexpr int MAX_BATCH = 16384;
constexpr int MAX_STEPS = 65536;
constexpr int LDH = WID + 8;     // LDS row pitch of the fused forward (BF16), 16 B skew per row

typedef uint16_t bf16_t;
typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f4 __attribute__((__vector_size__(4 * sizeof(float))));

// FP32 -> BF16, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ bf16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(bf16_t b) { return __uint_as_float((uint32_t)b << 16); }

// erfc(z) for z >= 0 by the Chebyshev fit of Press et al., Numerical Recipes
// (Sec. 6.2, erfcc): t exp(-z^2 + P(t)) with t = 1 / (1 + z/2), fractional
// error below 1.2e-7 in exact arithmetic (about 1e-6 in FP32 for z < 9).
__device__ __forceinline__ float erfc_pos(float z) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, z, 1.0f));
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  return t * __expf(fmaf(t, p, fmaf(-z, z, -1.26551223f)));
}
// 1 + erf(z): 2 - erfc(z) for z >= 0 and erfc(-z) below, so that the left
// tail keeps its relative precision (1 + erf(z) cancels there), which is what
// the BF16 rounding of the activation sees.
__device__ __forceinline__ float one_plus_erf(float z) {
  const float ec = erfc_pos(fabsf(z));
  return z >= 0.0f ? 2.0f - ec : ec;
}
// GELU(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2 and its derivative
// Phi(a) + a exp(-a^2/2) / sqrt(2 pi)
__device__ __forceinline__ float gelu(float a) { return 0.5f * a * one_plus_erf(a * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float a) {
  return 0.5f * one_plus_erf(a * 0.70710678118654752f) + a * 0.39894228040143268f * __expf(-0.5f * a * a);
}

__device__ __forceinline__ bf16x8 load8(const bf16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ f4 mma(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// normalisation constants on the device
struct Norm {
  float in_shift[NIN], in_scale[NIN], out_shift[NOUT], out_scale[NOUT], enc_freq[NIN];
};

// sin and cos of 2^k (p + e) for k = 0 .. K-1, where p + e is an angle held
// as an FP32 number and its rounding error: the octave doubles both exactly,
// and the first-order term 2^k e keeps the high octaves as accurate as the
// low ones (the rounding of the angle would otherwise grow with 2^k).
template <int K>
__device__ __forceinline__ void octaves(float p, float e, float* f) {
#pragma unroll
  for (int k = 0; k < K; ++k, p *= 2.0f, e *= 2.0f) {
    float s, c;
    sincosf(p, &s, &c);
    f[2 * k] = fmaf(e, c, s);
    f[2 * k + 1] = fmaf(-e, s, c);
  }
}

// The first layer's inputs of one raw row (x0, x1): the normalised inputs
// u_c, then sin and cos of 2^k enc_freq[c] u_c for the octaves of input 0,
// then those of input 1.
__device__ __forceinline__ void features(float x0, float x1, const Norm* nm, float* f) {
  const float u0 = (x0 - nm->in_shift[0]) * nm->in_scale[0];
  const float u1 = (x1 - nm->in_shift[1]) * nm->in_scale[1];
  f[0] = u0;
  f[1] = u1;
  const float p0 = nm->enc_freq[0] * u0, p1 = nm->enc_freq[1] * u1;
  octaves<NFQ0>(p0, fmaf(nm->enc_freq[0], u0, -p0), f + NIN);
  octaves<NFQ1>(p1, fmaf(nm->enc_freq[1], u1, -p1), f + NIN + 2 * NFQ0);
}

// ---------------------------------------------------------------------------
// training step, part 1: everything that is local to a batch row.  One block
// takes RB = 16 rows through the forward pass, the loss and the backward pass
// down to the input layer; the 16 x 256 activations and gradients stay in
// LDS between layers.  Sixteen waves; wave w owns hidden units 16w .. 16w+15
// (waves 0-3 also output units 16w .. 16w+15), so the thread that writes a
// pre-activation a_l[i][j] is the one that reads it back for GELU'(a_l) on
// the way down.  It writes what the
// weight-gradient products need (h_l^T, da_l^T, BF16) and per-block partial
// sums of the bias gradients, of the first layer's weight gradient and of the
// loss.
// ---------------------------------------------------------------------------
constexpr int RB = 16;          // batch rows per block of the fused step kernel
constexpr int LDY = NOUT + 8;   // LDS pitch of dL/dy (BF16)

struct RowArgs {
  const float* X;        // raw inputs [*][2], rows selected by `rows` (or the first n)
  const float* T;        // raw targets [*][NOUT]
  const int32_t* rows;
  int nvalid;            // rows >= nvalid are padding (zero gradient)
  float dscale;          // 2 / (nvalid * NOUT)
  const Norm* nm;
  const bf16_t *W1b, *W2b, *W3b, *W4b, *W2t, *W3t, *W4t;
  const float *b1, *b2, *b3, *b4;
  float *A1, *A2, *A3;              // FP32 pre-activations [Bp][WID]
  bf16_t *H1t, *H2t, *H3t;          // BF16 h_l^T [WID][ldt]
  bf16_t *DYt, *D3t, *D2t;          // BF16 dL/dy^T [NOUT][ldt], dL/da_l^T [WID][ldt]
  int ldt;
  float *bp1, *bp2, *bp3, *bp4;     // per-block bias-gradient columns [R][width]
  float* w1p;                       // per-block first-layer weight gradient [R][WID][NFEAT]
  double* lpart;                    // per-block sum of squared residuals [R]
};

// sum over the block's 16 rows of per-lane column values (lanes l, l^16, l^32,
// l^48 share a column); lanes 0..15 return the column sums
__device__ __forceinline__ float col_sum16(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// one 16 x (16 CT) slab of C = A Bt^T: A is the block's 16 rows in LDS (pitch
// lda), Bt rows col0 .. col0 + 16 CT - 1 in global memory (pitch ldb),
// K = 32 NK.  All weight fragments are requested before the first product, so
// the wave waits for memory once per layer instead of once per 32-deep step.
constexpr int CT = 1;  // 16-column tiles per wave
template <int NK>
__device__ __forceinline__ void slab16(const bf16_t* As, int lda, const bf16_t* __restrict__ Bt, int ldb,
                                       int col0, int lane, f4 (&acc)[CT]) {
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) acc[ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const bf16_t* pb = Bt + (size_t)(col0 + r16) * ldb + kq;
  bf16x8 b[NK][CT];
#pragma unroll
  for (int s = 0; s < NK; ++s)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) b[s][ct] = load8(pb + (size_t)ct * 16 * ldb + 32 * s);
  bf16x8 a[NK];
#pragma unroll
  for (int s = 0; s < NK; ++s) a[s] = load8(As + r16 * lda + 32 * s + kq);
  // keep the scheduler from sinking the loads back between the products
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s = 0; s < NK; ++s)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = mma(a[s], b[s][ct], acc[ct]);
}

__device__ __forceinline__ void store_t4(bf16_t* Ht, int j, int ldt, int i0, const bf16_t (&hb)[4]) {
  uint2 v;
  v.x = hb[0] | ((uint32_t)hb[1] << 16);
  v.y = hb[2] | ((uint32_t)hb[3] << 16);
  *reinterpret_cast<uint2*>(Ht + (size_t)j * ldt + i0) = v;
}

constexpr int NWAVE = WID / (16 * CT);       // 16
constexpr int L1R = RB * WID / (64 * NWAVE);  // layer-1 rows per thread (4)

__global__ __launch_bounds__(64 * NWAVE) void step_rows_kernel(RowArgs g) {
  __shared__ __align__(16) bf16_t HA[RB * LDH];
  __shared__ __align__(16) bf16_t HB[RB * LDH];
  __shared__ __align__(16) bf16_t DY[RB * LDY];
  __shared__ float xs[RB][NFEAT];
  __shared__ double lred[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rq = (lane >> 4) * 4;  // first of this lane's 4 rows in a 16-row tile
  const int rb = blockIdx.x, r0 = rb * RB;
  const int ldt = g.ldt;

  // layer 1 (K = NFEAT, plain FMA): thread t is unit t % 256 for L1R rows;
  // padding rows (past nvalid) take zero features
  if (t < RB) {
    const int i = r0 + t;
    if (i < g.nvalid) {
      const int64_t src = g.rows ? (int64_t)g.rows[i] : (int64_t)i;
      features(g.X[2 * src], g.X[2 * src + 1], g.nm, xs[t]);
    } else {
#pragma unroll
      for (int c = 0; c < NFEAT; ++c) xs[t][c] = 0.0f;
    }
  }
  __syncthreads();
  {
    const int j = t & (WID - 1), rh = (t / WID) * L1R;
    float wf[NFEAT];
#pragma unroll
    for (int c = 0; c < NFEAT; ++c) wf[c] = from_bf16(g.W1b[NFEAT * j + c]);
    const float bj = g.b1[j];
    uint32_t packed[L1R / 2];
#pragma unroll
    for (int q = 0; q < L1R; ++q) {
      const int r = rh + q;
      float a = bj;
#pragma unroll
      for (int c = 0; c < NFEAT; ++c) a = fmaf(xs[r][c], wf[c], a);
      const bf16_t hv = to_bf16(gelu(a));
      g.A1[(size_t)(r0 + r) * WID + j] = a;
      HA[r * LDH + j] = hv;
      if (q & 1) packed[q >> 1] |= (uint32_t)hv << 16;
      else packed[q >> 1] = hv;
    }
    static_assert(L1R == 4, "layer-1 rows per thread");
    *reinterpret_cast<uint2*>(g.H1t + (size_t)j * ldt + r0 + rh) = uint2{packed[0], packed[1]};
  }
  __syncthreads();

  // hidden layers 2 and 3: a = h W^T + b, h' = BF16(GELU(a))
  {
    const bf16_t* Wl[2] = {g.W2b, g.W3b};
    const float* bl[2] = {g.b2, g.b3};
    float* Al[2] = {g.A2, g.A3};
    bf16_t* Htl[2] = {g.H2t, g.H3t};
    bf16_t* src[2] = {HA, HB};
    bf16_t* dstb[2] = {HB, HA};
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      f4 acc[CT];
      slab16<WID / 32>(src[l], LDH, Wl[l], WID, 16 * CT * w, lane, acc);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int j = 16 * CT * w + 16 * ct + (lane & 15);
        const float bj = bl[l][j];
        bf16_t hb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = rq + e;
          const float a = acc[ct][e] + bj;
          Al[l][(size_t)(r0 + r) * WID + j] = a;
          hb[e] = to_bf16(gelu(a));
          dstb[l][r * LDH + j] = hb[e];
        }
        store_t4(Htl[l], j, ldt, r0 + rq, hb);
      }
      __syncthreads();
    }
  }

  // output layer, loss and dL/dy = 2 (y - t) / (n NOUT) in normalised units;
  // waves 0-3 own outputs 16w .. 16w+15
  if (w < NOUT / 16) {
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    f4 acc = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const bf16_t* pb = g.W4b + (size_t)(16 * w + r16) * WID + kq;
#pragma unroll
    for (int s = 0; s < WID / 32; ++s) acc = mma(load8(HA + r16 * LDH + 32 * s + kq), load8(pb + 32 * s), acc);
    // (8 independent 16-byte loads: the compiler issues them together)
    const int j = 16 * w + r16;
    const float bj = g.b4[j], sh = g.nm->out_shift[j], sc = g.nm->out_scale[j];
    double lsum = 0.0;
    float cs = 0.0f;
    bf16_t hb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = rq + e, i = r0 + r;
      const float y = acc[e] + bj;
      float dy = 0.0f;
      if (i < g.nvalid) {
        const int64_t src = g.rows ? (int64_t)g.rows[i] : (int64_t)i;
        const float tn = (g.T[src * NOUT + j] - sh) * sc;
        const float res = y - tn;
        lsum += (double)res * (double)res;
        dy = res * g.dscale;
      }
      hb[e] = to_bf16(dy);
      DY[r * LDY + j] = hb[e];
      cs += dy;
    }
    store_t4(g.DYt, j, ldt, r0 + rq, hb);
    cs = col_sum16(cs);
    if (lane < 16) g.bp4[(size_t)rb * NOUT + j] = cs;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) lsum += __shfl_xor(lsum, o);
    if (lane == 0) lred[w] = lsum;
  }
  static_assert(NOUT / 16 == 4, "loss partials of four waves");
  __syncthreads();
  if (t == 0) g.lpart[rb] = ((lred[0] + lred[1]) + lred[2]) + lred[3];

  // backward through layers 4 -> 3 -> 2 (da_l = (da_{l+1} W_{l+1}) GELU'(a_l)) and 2 -> 1
  {
    const bf16_t* Wt[3] = {g.W4t, g.W3t, g.W2t};
    const float* Al[3] = {g.A3, g.A2, g.A1};
    bf16_t* Dt[2] = {g.D3t, g.D2t};
    float* bp[3] = {g.bp3, g.bp2, g.bp1};
    const bf16_t* src[3] = {DY, HB, HA};
    const int lds[3] = {LDY, LDH, LDH};
    bf16_t* dstb[2] = {HB, HA};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      f4 acc[CT];
      if (l == 0) slab16<NOUT / 32>(src[l], lds[l], Wt[l], NOUT, 16 * CT * w, lane, acc);
      else slab16<WID / 32>(src[l], lds[l], Wt[l], WID, 16 * CT * w, lane, acc);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int j = 16 * CT * w + 16 * ct + (lane & 15);
        float c0 = 0.0f, dae[4];
        bf16_t hb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = rq + e;
          const float da = acc[ct][e] * gelu_grad(Al[l][(size_t)(r0 + r) * WID + j]);
          c0 += da;
          dae[e] = da;
          if (l < 2) {
            hb[e] = to_bf16(da);
            dstb[l][r * LDH + j] = hb[e];
          }
        }
        if (l < 2) store_t4(Dt[l], j, ldt, r0 + rq, hb);
        c0 = col_sum16(c0);
        if (lane < 16) bp[l][(size_t)rb * WID + j] = c0;
        if (l == 2) {
          // first layer's weight gradient: one feature at a time, summed
          // over the block's rows (rows e of this lane, then across lanes)
#pragma unroll
          for (int c = 0; c < NFEAT; ++c) {
            float cf = 0.0f;
#pragma unroll
            for (int e = 0; e < 4; ++e) cf = fmaf(dae[e], xs[rq + e][c], cf);
            cf = col_sum16(cf);
            if (lane < 16) g.w1p[((size_t)rb * WID + j) * NFEAT + c] = cf;
          }
        }
      }
      if (l < 2) __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// training step, part 2: the three weight-gradient products
//   gW_l[M][N] = sum over batch rows of da_l^T h_{l-1}  (A = da_l^T, Bt = h_{l-1}^T)
// in one launch, each split over KSPLIT batch rows into its own partial slab
// (summed in split order by the finishing kernel).  64 x 64 block tiles, four
// waves of 32 x 32; all operand fragments of a block are loaded first.
// ---------------------------------------------------------------------------
struct WgradProduct {
  const bf16_t* A;   // [M][K], pitch ld
  const bf16_t* Bt;  // [N][K], pitch ld
  float* part;       // [splits][M][N]
  int M;
};

struct WgradArgs {
  WgradProduct p[3];
  int ld, K, S;      // pitch (= max batch), batch rows, splits
  int first[4];      // first block of each product (cumulative)
};

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs g) {
  const int b = blockIdx.x;
  const int pi = b < g.first[1] ? 0 : (b < g.first[2] ? 1 : 2);
  const WgradProduct& P = g.p[pi];
  constexpr int N = WID, TX = WID / 64;
  const int ty = P.M / 64, loc = b - g.first[pi];
  const int bx = loc % TX, by = (loc / TX) % ty, bz = loc / (TX * ty);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const int row0 = by * 64 + wr * 32, col0 = bx * 64 + wc * 32;
  const int kb = bz * KSPLIT, ke = min(g.K, kb + KSPLIT);
  const int nk = (ke - kb) >> 5;  // 2, 4, 6 or 8
  const bf16_t* pa0 = P.A + (size_t)(row0 + r16) * g.ld + kq;
  const bf16_t* pa1 = pa0 + (size_t)16 * g.ld;
  const bf16_t* pb0 = P.Bt + (size_t)(col0 + r16) * g.ld + kq;
  const bf16_t* pb1 = pb0 + (size_t)16 * g.ld;
  f4 acc[2][2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  bf16x8 fa[8][2], fb[8][2];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    if (s < nk) {
      const int k = kb + 32 * s;
      fa[s][0] = load8(pa0 + k);
      fa[s][1] = load8(pa1 + k);
      fb[s][0] = load8(pb0 + k);
      fb[s][1] = load8(pb1 + k);
    }
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    if (s < nk) {
      acc[0][0] = mma(fa[s][0], fb[s][0], acc[0][0]);
      acc[0][1] = mma(fa[s][0], fb[s][1], acc[0][1]);
      acc[1][0] = mma(fa[s][1], fb[s][0], acc[1][0]);
      acc[1][1] = mma(fa[s][1], fb[s][1], acc[1][1]);
    }
  }
  float* out = P.part + (size_t)bz * P.M * N;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = row0 + rt * 16 + (lane >> 4) * 4 + e, j = col0 + ct * 16 + r16;
        out[(size_t)i * N + j] = acc[rt][ct][e];
      }
}

// ---------------------------------------------------------------------------
// gradient assembly (fixed-order sums of the partials) and Adam
// ---------------------------------------------------------------------------
struct WCopies {
  bf16_t *W1b, *W2b, *W2t, *W3b, *W3t, *W4b, *W4t;
};

__device__ __forceinline__ void store_copies(int p, float v, const WCopies& c) {
  const bf16_t b = to_bf16(v);
  if (p < OB1) {
    c.W1b[p] = b;
  } else if (p >= OW2 && p < OB2) {
    const int e = p - OW2, o = e / WID, i = e % WID;
    c.W2b[e] = b;
    c.W2t[i * WID + o] = b;
  } else if (p >= OW3 && p < OB3) {
    const int e = p - OW3, o = e / WID, i = e % WID;
    c.W3b[e] = b;
    c.W3t[i * WID + o] = b;
  } else if (p >= OW4 && p < OB4) {
    const int e = p - OW4, o = e / WID, i = e % WID;
    c.W4b[e] = b;
    c.W4t[i * NOUT + o] = b;
  }
}

__global__ __launch_bounds__(256) void copies_kernel(const float* __restrict__ P, WCopies c) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < NPAR) store_copies(p, P[p], c);
}

// Training control on the device, so that a captured epoch can be replayed:
// the learning rate of the epoch and the number of Adam steps taken before it.
struct TrainCtl {
  double t0;
  double lr;
};

struct FinishArgs {
  const float *part2, *part3, *part4, *bp1, *bp2, *bp3, *bp4, *w1p;
  const double* lpart;
  int S, R;            // splits of the weight products, RB-row blocks
  double inv_count;    // 1 / (nvalid * 64)
  double* loss;        // one FP64
  float* G;            // gradient out [NPAR]
  // Adam: step t = ctl->t0 + step + 1, bias corrections 1 - beta^t
  float *P, *Mo, *Ve;
  const TrainCtl* ctl;
  int step;
  double beta1, beta2;
  float eps;
  WCopies c;
};

__global__ void ctl_set_lr(TrainCtl* c, double lr) {
  if (threadIdx.x == 0) c->lr = lr;
}
__global__ void ctl_advance(TrainCtl* c, int nsteps) {
  if (threadIdx.x == 0) c->t0 += (double)nsteps;
}

// sum_{r < n} base[r * stride] in order r = 0, 1, ...; the loads are issued
// 16 at a time so that the chain waits for memory once per 16 terms
__device__ __forceinline__ float ordered_sum(const float* __restrict__ base, size_t stride, int n) {
  float g = 0.0f;
  for (int r0 = 0; r0 < n; r0 += 16) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (r0 + k < n) ? base[(size_t)(r0 + k) * stride] : 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (r0 + k < n) g += v[k];
  }
  return g;
}

template <bool UPDATE>
__global__ __launch_bounds__(256) void finish_kernel(FinishArgs f) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p == 0) {
    double s = 0.0;
    for (int r = 0; r < f.R; ++r) s += f.lpart[r];
    f.loss[0] = s * f.inv_count;
  }
  if (p >= NPAR) return;
  float g;
  if (p < OB1) {
    const int j = p / NFEAT, c = p % NFEAT;
    g = ordered_sum(f.w1p + (size_t)j * NFEAT + c, (size_t)WID * NFEAT, f.R);
  } else if (p < OW2) {
    g = ordered_sum(f.bp1 + (p - OB1), WID, f.R);
  } else if (p < OB2) {
    g = ordered_sum(f.part2 + (p - OW2), (size_t)WID * WID, f.S);
  } else if (p < OW3) {
    g = ordered_sum(f.bp2 + (p - OB2), WID, f.R);
  } else if (p < OB3) {
    g = ordered_sum(f.part3 + (p - OW3), (size_t)WID * WID, f.S);
  } else if (p < OW4) {
    g = ordered_sum(f.bp3 + (p - OB3), WID, f.R);
  } else if (p < OB4) {
    g = ordered_sum(f.part4 + (p - OW4), (size_t)NOUT * WID, f.S);
  } else {
    g = ordered_sum(f.bp4 + (p - OB4), NOUT, f.R);
  }
  f.G[p] = g;
  if constexpr (UPDATE) {
    const double t = f.ctl->t0 + (double)(f.step + 1);
    const float bc1 = (float)(1.0 - pow(f.beta1, t)), bc2 = (float)(1.0 - pow(f.beta2, t));
    const float lr = (float)f.ctl->lr, b1 = (float)f.beta1, b2 = (float)f.beta2;
    const float m = b1 * f.Mo[p] + (1.0f - b1) * g;
    const float v = b2 * f.Ve[p] + (1.0f - b2) * g * g;
    f.Mo[p] = m;
    f.Ve[p] = v;
    const float w = f.P[p] - lr * (m / bc1) / (sqrtf(v / bc2) + f.eps);
    f.P[p] = w;
    store_copies(p, w, f.c);
  }
}

// ---------------------------------------------------------------------------
// fused inference: 64 query rows per block, activations stay in LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void predict_kernel(const float* __restrict__ X, int64_t n,
                                                      const Norm* __restrict__ nm, const bf16_t* __restrict__ W1b,
                                                      const float* __restrict__ b1, const bf16_t* __restrict__ W2b,
                                                      const float* __restrict__ b2, const bf16_t* __restrict__ W3b,
                                                      const float* __restrict__ b3, const bf16_t* __restrict__ W4b,
                                                      const float* __restrict__ b4, float* __restrict__ Y) {
  __shared__ __align__(16) bf16_t H[64 * LDH];
  __shared__ float xs[64][NFEAT];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  if (t < 64) {
    const int64_t i = r0 + t;
    if (i < n) {
      features(X[2 * i], X[2 * i + 1], nm, xs[t]);
    } else {
#pragma unroll
      for (int c = 0; c < NFEAT; ++c) xs[t][c] = 0.0f;
    }
  }
  __syncthreads();
  {
    const int j = t;
    float wf[NFEAT];
#pragma unroll
    for (int c = 0; c < NFEAT; ++c) wf[c] = from_bf16(W1b[NFEAT * j + c]);
    const float bj = b1[j];
    for (int r = 0; r < 64; ++r) {
      float a = bj;
#pragma unroll
      for (int c = 0; c < NFEAT; ++c) a = fmaf(xs[r][c], wf[c], a);
      H[r * LDH + j] = to_bf16(gelu(a));
    }
  }
  __syncthreads();
  // hidden layers 2 and 3: wave w owns columns 64w .. 64w+63 of all 64 rows
  for (int layer = 0; layer < 2; ++layer) {
    const bf16_t* W = layer ? W3b : W2b;
    const float* bias = layer ? b3 : b2;
    f4 acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const bf16_t* wb = W + (size_t)(64 * w + r16) * WID + kq;
#pragma unroll 2
    for (int kk = 0; kk < WID; kk += 32) {
      bf16x8 a[4], b[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) b[ct] = load8(wb + (size_t)ct * 16 * WID + kk);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) a[rt] = load8(&H[(rt * 16 + r16) * LDH + kk + kq]);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mma(a[rt], b[ct], acc[rt][ct]);
    }
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int j = 64 * w + ct * 16 + r16;
      const float bj = bias[j];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          H[(rt * 16 + (lane >> 4) * 4 + e) * LDH + j] = to_bf16(gelu(acc[rt][ct][e] + bj));
    }
    __syncthreads();
  }
  // output layer: wave w owns columns 16w .. 16w+15
  f4 acc[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc[rt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const bf16_t* wb = W4b + (size_t)(16 * w + r16) * WID + kq;
#pragma unroll 2
  for (int kk = 0; kk < WID; kk += 32) {
    const bf16x8 b = load8(wb + kk);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) acc[rt] = mma(load8(&H[(rt * 16 + r16) * LDH + kk + kq]), b, acc[rt]);
  }
  const int j = 16 * w + r16;
  const float bj = b4[j], sh = nm->out_shift[j], sc = nm->out_scale[j];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = r0 + rt * 16 + (lane >> 4) * 4 + e;
      if (i < n) Y[i * NOUT + j] = (acc[rt][e] + bj) / sc + sh;
    }
}

}  // namespace

// per-column mean and 1/std of the targets (one block per column, FP64,
// fixed-order tree reduction)
__global__ __launch_bounds__(256) void column_stats(const float* __restrict__ T, int64_t n, Norm* nm,
                                                    double* out) {
  __shared__ double red[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < n; i += 256) s += (double)T[i * NOUT + c];
  red[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (int64_t i = t; i < n; i += 256) {
    const double d = (double)T[i * NOUT + c] - mean;
    q += d * d;
  }
  red[t] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) {
    const double sd = fmax(sqrt(red[0] / (double)n), 1e-6);
    out[c] = mean;
    out[NOUT + c] = 1.0 / sd;
    nm->out_shift[c] = (float)mean;
    nm->out_scale[c] = (float)(1.0 / sd);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct surrogate_t {
  surrogate_params p;
  hipStream_t stream;
  int B;  // max_batch
  float *P, *Mo, *Ve, *G, *A1, *A2, *A3;
  Norm* nm;
  WCopies wc;
  bf16_t *H1t, *H2t, *H3t, *DYt, *D3t, *D2t;
  float *part2, *part3, *part4, *bp1, *bp2, *bp3, *bp4, *w1p;
  double *lpart, *losses, *stats;
  TrainCtl* ctl;
  int64_t t;   // Adam steps taken
  bool loaded;
  // captured epoch, replayed while its inputs are the same buffers and sizes
  bool use_graph;
  hipGraphExec_t graph;
  const void* gkey[3];
  int64_t gn;
};

namespace {

// carve the workspace (base == nullptr: only measure)
size_t carve(int B, char* base, surrogate_t* s) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~(size_t)255;
    char* q = base ? base + off : nullptr;
    off += bytes;
    return q;
  };
  const int S = (B + KSPLIT - 1) / KSPLIT, R = B / RB;
  surrogate_t d{};
  surrogate_t& h = s ? *s : d;
  h.P = (float*)take(4ull * NPAR);
  h.Mo = (float*)take(4ull * NPAR);
  h.Ve = (float*)take(4ull * NPAR);
  h.G = (float*)take(4ull * NPAR);
  h.nm = (Norm*)take(sizeof(Norm));
  h.wc.W1b = (bf16_t*)take(2ull * WID * NFEAT);
  h.wc.W2b = (bf16_t*)take(2ull * WID * WID);
  h.wc.W2t = (bf16_t*)take(2ull * WID * WID);
  h.wc.W3b = (bf16_t*)take(2ull * WID * WID);
  h.wc.W3t = (bf16_t*)take(2ull * WID * WID);
  h.wc.W4b = (bf16_t*)take(2ull * NOUT * WID);
  h.wc.W4t = (bf16_t*)take(2ull * NOUT * WID);
  h.A1 = (float*)take(4ull * B * WID);
  h.A2 = (float*)take(4ull * B * WID);
  h.A3 = (float*)take(4ull * B * WID);
  bf16_t** act[] = {&h.H1t, &h.H2t, &h.H3t, &h.D3t, &h.D2t};
  for (bf16_t** a : act) *a = (bf16_t*)take(2ull * B * WID);
  h.DYt = (bf16_t*)take(2ull * B * NOUT);
  h.part2 = (float*)take(4ull * S * WID * WID);
  h.part3 = (float*)take(4ull * S * WID * WID);
  h.part4 = (float*)take(4ull * S * NOUT * WID);
  h.bp1 = (float*)take(4ull * R * WID);
  h.bp2 = (float*)take(4ull * R * WID);
  h.bp3 = (float*)take(4ull * R * WID);
  h.bp4 = (float*)take(4ull * R * NOUT);
  h.w1p = (float*)take(4ull * R * WID * NFEAT);
  h.lpart = (double*)take(8ull * R);
  h.losses = (double*)take(8ull * MAX_STEPS);
  h.stats = (double*)take(8ull * 2 * NOUT);
  h.ctl = (TrainCtl*)take(sizeof(TrainCtl));
  return off + 256;
}

int validate(const surrogate_params* p) {
  if (!p) { set_error("NULL params"); return LAT_EINVAL; }
  if (p->max_batch < 64 || p->max_batch > MAX_BATCH || p->max_batch % 64) {
    set_error("max_batch must be a multiple of 64 in [64, 16384]");
    return LAT_EINVAL;
  }
  if (!(p->beta1 >= 0.0 && p->beta1 < 1.0 && p->beta2 >= 0.0 && p->beta2 < 1.0 && p->eps > 0.0)) {
    set_error("Adam parameters: need 0 <= beta < 1 and eps > 0");
    return LAT_EINVAL;
  }
  for (int c = 0; c < NIN; ++c)
    if (!std::isfinite(p->in_shift[c]) || !std::isfinite(p->in_scale[c]) || p->in_scale[c] == 0.0f ||
        !std::isfinite(p->enc_freq[c])) {
      set_error("input normalisation must be finite with nonzero scale, and the encoding frequencies finite");
      return LAT_EINVAL;
    }
  for (int c = 0; c < NOUT; ++c)
    if (!std::isfinite(p->out_shift[c]) || !std::isfinite(p->out_scale[c]) || p->out_scale[c] == 0.0f) {
      set_error("output normalisation must be finite with nonzero scale");
      return LAT_EINVAL;
    }
  return LAT_OK;
}

void drop_graph(surrogate_t* h) {
  if (h->graph) hipGraphExecDestroy(h->graph);
  h->graph = nullptr;
  h->gkey[0] = h->gkey[1] = h->gkey[2] = nullptr;
  h->gn = 0;
}

// forward + backward of n rows (rows[] may be NULL) into G, loss into *loss_dev;
// with update, one Adam step on the master weights and their BF16 copies
int train_step(surrogate_t* h, const float* X, const float* T, const int32_t* rows, int n, float* G,
               double* loss_dev, bool update, int step) {
  hipStream_t st = h->stream;
  const int Bp = (n + 63) / 64 * 64, R = Bp / RB, S = (Bp + KSPLIT - 1) / KSPLIT, ldt = h->B;
  const WCopies& c = h->wc;
  // rows: forward, loss, backward to the input layer
  RowArgs ra{};
  ra.X = X; ra.T = T; ra.rows = rows; ra.nvalid = n;
  ra.dscale = (float)(2.0 / ((double)n * NOUT));
  ra.nm = h->nm;
  ra.W1b = c.W1b; ra.W2b = c.W2b; ra.W3b = c.W3b; ra.W4b = c.W4b;
  ra.W2t = c.W2t; ra.W3t = c.W3t; ra.W4t = c.W4t;
  ra.b1 = h->P + OB1; ra.b2 = h->P + OB2; ra.b3 = h->P + OB3; ra.b4 = h->P + OB4;
  ra.A1 = h->A1; ra.A2 = h->A2; ra.A3 = h->A3;
  ra.H1t = h->H1t; ra.H2t = h->H2t; ra.H3t = h->H3t;
  ra.DYt = h->DYt; ra.D3t = h->D3t; ra.D2t = h->D2t;
  ra.ldt = ldt;
  ra.bp1 = h->bp1; ra.bp2 = h->bp2; ra.bp3 = h->bp3; ra.bp4 = h->bp4;
  ra.w1p = h->w1p; ra.lpart = h->lpart;
  hipLaunchKernelGGL(step_rows_kernel, dim3(R), dim3(64 * NWAVE), 0, st, ra);
  CL_HIP(hipGetLastError());
  // weight gradients of layers 4, 3, 2
  WgradArgs wa{};
  wa.p[0] = WgradProduct{h->DYt, h->H3t, h->part4, NOUT};
  wa.p[1] = WgradProduct{h->D3t, h->H2t, h->part3, WID};
  wa.p[2] = WgradProduct{h->D2t, h->H1t, h->part2, WID};
  wa.ld = ldt; wa.K = Bp; wa.S = S;
  wa.first[0] = 0;
  for (int q = 0; q < 3; ++q) wa.first[q + 1] = wa.first[q] + (WID / 64) * (wa.p[q].M / 64) * S;
  hipLaunchKernelGGL(wgrad_kernel, dim3(wa.first[3]), dim3(256), 0, st, wa);
  CL_HIP(hipGetLastError());
  FinishArgs f{};
  f.part2 = h->part2; f.part3 = h->part3; f.part4 = h->part4;
  f.bp1 = h->bp1; f.bp2 = h->bp2; f.bp3 = h->bp3; f.bp4 = h->bp4; f.w1p = h->w1p;
  f.lpart = h->lpart; f.S = S; f.R = R;
  f.inv_count = 1.0 / ((double)n * NOUT);
  f.loss = loss_dev;
  f.G = G;
  f.P = h->P; f.Mo = h->Mo; f.Ve = h->Ve;
  f.c = c;
  const int fb = (NPAR + 255) / 256;
  if (update) {
    f.ctl = h->ctl;
    f.step = step;
    f.beta1 = h->p.beta1;
    f.beta2 = h->p.beta2;
    f.eps = (float)h->p.eps;
    hipLaunchKernelGGL(finish_kernel<true>, dim3(fb), dim3(256), 0, st, f);
  } else {
    hipLaunchKernelGGL(finish_kernel<false>, dim3(fb), dim3(256), 0, st, f);
  }
  CL_HIP(hipGetLastError());
  return LAT_OK;
}

}  // namespace

extern "C" int surrogate_workspace_size(const surrogate_params* p, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes) { set_error("NULL argument"); return LAT_EINVAL; }
  *bytes = carve(p->max_batch, nullptr, nullptr);
  return LAT_OK;
}

extern "C" int surrogate_init(const surrogate_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                              surrogate_t** out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!dev_ws || !out) { set_error("NULL argument"); return LAT_EINVAL; }
  const size_t need = carve(p->max_batch, nullptr, nullptr);
  if (ws_bytes < need) { set_error("workspace too small: need " + std::to_string(need)); return LAT_ENOMEM; }
  surrogate_t* h = new (std::nothrow) surrogate_t{};
  if (!h) { set_error("out of host memory"); return LAT_ENOMEM; }
  h->p = *p;
  h->stream = (hipStream_t)hip_stream;
  h->B = p->max_batch;
  h->use_graph = hip_stream != nullptr;
  char* base = (char*)(((uintptr_t)dev_ws + 255) & ~(uintptr_t)255);
  carve(h->B, base, h);
  Norm nm;
  std::memcpy(nm.in_shift, p->in_shift, sizeof nm.in_shift);
  std::memcpy(nm.in_scale, p->in_scale, sizeof nm.in_scale);
  std::memcpy(nm.out_shift, p->out_shift, sizeof nm.out_shift);
  std::memcpy(nm.out_scale, p->out_scale, sizeof nm.out_scale);
  std::memcpy(nm.enc_freq, p->enc_freq, sizeof nm.enc_freq);
  hipError_t e = hipMemcpyAsync(h->nm, &nm, sizeof(Norm), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    set_error(std::string("surrogate_init: ") + hipGetErrorString(e));
    delete h;
    return LAT_EHIP;
  }
  *out = h;
  return LAT_OK;
}

extern "C" int surrogate_set_weights(surrogate_t* h, const float* host_w) {
  if (!h || !host_w) { set_error("NULL argument"); return LAT_EINVAL; }
  for (int i = 0; i < NPAR; ++i)
    if (!std::isfinite(host_w[i])) { set_error("non-finite weight"); return LAT_EINVAL; }
  CL_HIP(hipMemcpyAsync(h->P, host_w, 4ull * NPAR, hipMemcpyHostToDevice, h->stream));
  CL_HIP(hipMemsetAsync(h->Mo, 0, 4ull * NPAR, h->stream));
  CL_HIP(hipMemsetAsync(h->Ve, 0, 4ull * NPAR, h->stream));
  CL_HIP(hipMemsetAsync(h->ctl, 0, sizeof(TrainCtl), h->stream));
  hipLaunchKernelGGL(copies_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, h->stream, h->P, h->wc);
  CL_HIP(hipGetLastError());
  CL_HIP(hipStreamSynchronize(h->stream));
  h->t = 0;
  h->loaded = true;
  return LAT_OK;
}

extern "C" int surrogate_get_weights(surrogate_t* h, float* host_w) {
  if (!h || !host_w) { set_error("NULL argument"); return LAT_EINVAL; }
  if (!h->loaded) { set_error("weights not set"); return LAT_ESTATE; }
  CL_HIP(hipMemcpyAsync(host_w, h->P, 4ull * NPAR, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipStreamSynchronize(h->stream));
  return LAT_OK;
}

extern "C" int surrogate_fit_output_scale(surrogate_t* h, const float* dev_t, int64_t n, double* host_shift,
                                          double* host_scale) {
  if (!h || !dev_t) { set_error("NULL argument"); return LAT_EINVAL; }
  if (n < 2) { set_error("need at least 2 target rows"); return LAT_EINVAL; }
  hipLaunchKernelGGL(column_stats, dim3(NOUT), dim3(256), 0, h->stream, dev_t, n, h->nm, h->stats);
  CL_HIP(hipGetLastError());
  double st[2 * NOUT];
  CL_HIP(hipMemcpyAsync(st, h->stats, sizeof st, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipStreamSynchronize(h->stream));
  for (int c = 0; c < 2 * NOUT; ++c)
    if (!std::isfinite(st[c])) { set_error("non-finite target statistics"); return LAT_ENONFINITE; }
  for (int c = 0; c < NOUT; ++c) {
    h->p.out_shift[c] = (float)st[c];
    h->p.out_scale[c] = (float)st[NOUT + c];
    if (host_shift) host_shift[c] = st[c];
    if (host_scale) host_scale[c] = st[NOUT + c];
  }
  return LAT_OK;
}

extern "C" int surrogate_loss_grad(surrogate_t* h, const float* dev_x, const float* dev_t, const int32_t* rows,
                                   int32_t n, float* dev_grad, double* loss) {
  if (!h || !dev_x || !dev_t || !dev_grad || !loss) { set_error("NULL argument"); return LAT_EINVAL; }
  if (!h->loaded) { set_error("weights not set"); return LAT_ESTATE; }
  if (n < 1 || n > h->B) { set_error("n must be in [1, max_batch]"); return LAT_EINVAL; }
  int rc = train_step(h, dev_x, dev_t, rows, n, dev_grad, h->losses, false, 0);
  if (rc) return rc;
  CL_HIP(hipMemcpyAsync(loss, h->losses, 8, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipStreamSynchronize(h->stream));
  if (!std::isfinite(*loss)) { set_error("non-finite loss"); return LAT_ENONFINITE; }
  return LAT_OK;
}

extern "C" int surrogate_train_epoch(surrogate_t* h, const float* dev_x, const float* dev_t,
                                     const int32_t* dev_perm, int64_t n, double lr, double* mean_loss) {
  if (!h || !dev_x || !dev_t || !dev_perm || !mean_loss) { set_error("NULL argument"); return LAT_EINVAL; }
  if (!h->loaded) { set_error("weights not set"); return LAT_ESTATE; }
  if (n < 1) { set_error("n must be positive"); return LAT_EINVAL; }
  if (!(lr > 0.0) || !std::isfinite(lr)) { set_error("lr must be positive"); return LAT_EINVAL; }
  const int64_t steps = (n + h->B - 1) / h->B;
  if (steps > MAX_STEPS) { set_error("too many steps in one epoch (max 65536)"); return LAT_EINVAL; }
  hipLaunchKernelGGL(ctl_set_lr, dim3(1), dim3(64), 0, h->stream, h->ctl, lr);
  CL_HIP(hipGetLastError());
  auto record = [&]() -> int {
    for (int64_t s = 0; s < steps; ++s) {
      const int ns = (int)std::min<int64_t>(h->B, n - s * h->B);
      int rc = train_step(h, dev_x, dev_t, dev_perm + s * h->B, ns, h->G, h->losses + s, true, (int)s);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(ctl_advance, dim3(1), dim3(64), 0, h->stream, h->ctl, (int)steps);
    CL_HIP(hipGetLastError());
    return LAT_OK;
  };
  const bool same = h->graph && h->gkey[0] == dev_x && h->gkey[1] == dev_t && h->gkey[2] == dev_perm && h->gn == n;
  if (h->use_graph && !same) {
    drop_graph(h);
    CL_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    const int rc = record();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    CL_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) {
      h->graph = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
      return LAT_EHIP;
    }
    h->gkey[0] = dev_x;
    h->gkey[1] = dev_t;
    h->gkey[2] = dev_perm;
    h->gn = n;
  }
  if (h->use_graph) {
    CL_HIP(hipGraphLaunch(h->graph, h->stream));
  } else {
    const int rc = record();
    if (rc) return rc;
  }
  h->t += steps;
  std::vector<double> l((size_t)steps);
  CL_HIP(hipMemcpyAsync(l.data(), h->losses, 8 * steps, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipStreamSynchronize(h->stream));
  double m = 0.0;
  for (double v : l) m += v;
  *mean_loss = m / (double)steps;
  if (!std::isfinite(*mean_loss)) { set_error("non-finite loss"); return LAT_ENONFINITE; }
  return LAT_OK;
}

extern "C" int surrogate_predict(surrogate_t* h, const float* dev_x, int64_t n, float* dev_y) {
  if (!h || !dev_x || !dev_y) { set_error("NULL argument"); return LAT_EINVAL; }
  if (!h->loaded) { set_error("weights not set"); return LAT_ESTATE; }
  if (n < 0 || n > ((int64_t)1 << 36)) { set_error("n out of range"); return LAT_EINVAL; }
  if (n == 0) return LAT_OK;
  const WCopies& c = h->wc;
  hipLaunchKernelGGL(predict_kernel, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, h->stream, dev_x, n, h->nm,
                     c.W1b, h->P + OB1, c.W2b, h->P + OB2, c.W3b, h->P + OB3, c.W4b, h->P + OB4, dev_y);
  CL_HIP(hipGetLastError());
  return LAT_OK;
}

extern "C" int surrogate_use_graph(surrogate_t* h, int on) {
  if (!h) { set_error("NULL handle"); return LAT_EINVAL; }
  if (on && !h->stream) { set_error("graph capture needs a created (non-default) stream"); return LAT_EINVAL; }
  CL_HIP(hipStreamSynchronize(h->stream));
  drop_graph(h);
  h->use_graph = on != 0;
  return LAT_OK;
}

extern "C" int surrogate_destroy(surrogate_t* h) {
  if (!h) return LAT_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  drop_graph(h);
  delete h;
  if (e != hipSuccess) { set_error(std::string("surrogate_destroy: ") + hipGetErrorString(e)); return LAT_EHIP; }
  return LAT_OK;
}
