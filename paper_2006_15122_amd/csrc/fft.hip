// Discrete Fourier transforms, binned power spectra and initial conditions.
//
// DFT convention (Sec. 3.1): f(n~) = sum_n e^{+2 pi i n~.n/N} f(n),
// f(n) = N^-3 sum_n~ e^{-2 pi i n~.n/N} f(n~).
// The 3-D transform is three passes of batched 1-D mixed-radix Stockham FFTs,
// one per axis; a block holds a batch of lines in LDS (ping-pong) and runs
// every radix stage there, so each pass reads and writes HBM once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace cl {

// complex number; 2 sizeof(R) alignment lets one 16-byte access move an FP64
// value (LDS and HBM)
template <typename R>
struct alignas(2 * sizeof(R)) Cx {
  R x, y;
};

struct FFTPlan {
  int N;
  int nfac;
  int fac[16];
};

// Factors of N: radix 8 first where r8 (the binning pass), then 4, 2 and
// odd primes.
static FFTPlan make_plan(int N, bool r8 = false) {
  FFTPlan P;
  P.N = N;
  P.nfac = 0;
  int n = N;
  if (r8)
    while (n % 8 == 0 && n != 16) { P.fac[P.nfac++] = 8; n /= 8; }
  while (n % 4 == 0) { P.fac[P.nfac++] = 4; n /= 4; }
  while (n % 2 == 0) { P.fac[P.nfac++] = 2; n /= 2; }
  for (int p = 3; n > 1; p += 2)
    while (n % p == 0) { P.fac[P.nfac++] = p; n /= p; }
  return P;
}

constexpr int kMaxRadix = 32;

template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return Cx<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Table of the N-th roots of unity W[m] = e^{+2 pi i m/N} (FP64), built once per
// lattice; the inverse transform uses their conjugates.
__global__ void twiddle_kernel(Cx<double>* W, int N) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) {
    double sv, cv;
    sincospi(2.0 * (double)m / (double)N, &sv, &cv);
    W[m] = Cx<double>{cv, sv};
  }
}

// Root W[q] (conjugated for sg < 0).  PAD: the table is the LDS copy, with
// one entry of padding after every 16 (the lanes of a stage read roots at
// strides that are multiples of 16 entries).
template <typename R, bool PAD = false>
__device__ __forceinline__ Cx<R> twiddle(const Cx<double>* __restrict__ W, int q, double sg) {
  const Cx<double> w = W[PAD ? q + (q >> 4) : q];
  return Cx<R>{(R)w.x, (R)(sg * w.y)};
}

// Length-RAD DFT o[m] = sum_r v[r] e^{sgn 2 pi i r m / RAD}; radices 2 and 4
// in closed form, others with roots from the table (index r m N/RAD mod N).
template <typename R, int RAD, bool PAD = false>
__device__ __forceinline__ void small_dft(const Cx<R>* v, Cx<R>* o, const Cx<double>* __restrict__ W, int N,
                                          double sg) {
  if constexpr (RAD == 2) {
    o[0] = Cx<R>{v[0].x + v[1].x, v[0].y + v[1].y};
    o[1] = Cx<R>{v[0].x - v[1].x, v[0].y - v[1].y};
  } else if constexpr (RAD == 4) {
    // e^{sgn 2 pi i m r/4}: multiplication by sgn*i for m r = 1 (mod 4)
    const R s = (R)sg;
    const Cx<R> a0{v[0].x + v[2].x, v[0].y + v[2].y}, a1{v[0].x - v[2].x, v[0].y - v[2].y};
    const Cx<R> b0{v[1].x + v[3].x, v[1].y + v[3].y}, b1{v[1].x - v[3].x, v[1].y - v[3].y};
    o[0] = Cx<R>{a0.x + b0.x, a0.y + b0.y};
    o[2] = Cx<R>{a0.x - b0.x, a0.y - b0.y};
    o[1] = Cx<R>{a1.x - s * b1.y, a1.y + s * b1.x};
    o[3] = Cx<R>{a1.x + s * b1.y, a1.y - s * b1.x};
  } else if constexpr (RAD == 8) {
    // 8 = 2 x 4 with r = r2 + 2 r1 and m = m1 + 4 m2: length-4 DFTs of the
    // even and the odd inputs, the odd ones times e^{sgn 2 pi i m1/8}, then
    // o[m1] and o[m1 + 4] as their sum and difference
    const R s = (R)sg, hf = (R)0.70710678118654752440084436210484904;
    const Cx<R> ev[4] = {v[0], v[2], v[4], v[6]}, od[4] = {v[1], v[3], v[5], v[7]};
    Cx<R> a[4], b[4];
    small_dft<R, 4>(ev, a, W, N, sg);
    small_dft<R, 4>(od, b, W, N, sg);
    b[1] = Cx<R>{hf * (b[1].x - s * b[1].y), hf * (b[1].y + s * b[1].x)};
    b[2] = Cx<R>{-s * b[2].y, s * b[2].x};
    b[3] = Cx<R>{-hf * (b[3].x + s * b[3].y), hf * (s * b[3].x - b[3].y)};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      o[m] = Cx<R>{a[m].x + b[m].x, a[m].y + b[m].y};
      o[m + 4] = Cx<R>{a[m].x - b[m].x, a[m].y - b[m].y};
    }
  } else {
#pragma unroll
    for (int m = 0; m < RAD; ++m) {
      double sx = (double)v[0].x, sy = (double)v[0].y;
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        const Cx<R> w = twiddle<R, PAD>(W, ((r * m) % RAD) * (N / RAD), sg);
        sx += (double)v[r].x * (double)w.x - (double)v[r].y * (double)w.y;
        sy += (double)v[r].x * (double)w.y + (double)v[r].y * (double)w.x;
      }
      o[m] = Cx<R>{(R)sx, (R)sy};
    }
  }
}

// One Stockham stage of radix RAD over B lines of length N held in LDS
// (in -> out); Ns is the length of the sub-transforms already done.
template <typename R, int RAD>
__device__ __forceinline__ void fft_stage(const Cx<R>* in, Cx<R>* out, const Cx<double>* __restrict__ W, int N,
                                          int B, int Ns, double sg) {
  const int M = N / RAD;
  const int stride = N / (Ns * RAD);  // k r stride < N for k < Ns, r < RAD
  for (int t = threadIdx.x; t < B * M; t += blockDim.x) {
    const int b = t / M, j = t - b * M, k = j % Ns;
    Cx<R> v[RAD], o[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      Cx<R> x = in[b * N + j + r * M];
      if (r > 0 && k > 0) x = cmul(x, twiddle<R>(W, k * r * stride, sg));
      v[r] = x;
    }
    small_dft<R, RAD>(v, o, W, N, sg);
    const int idxD = (j / Ns) * Ns * RAD + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) out[b * N + idxD + r * Ns] = o[r];
  }
}

// Stage of any radix up to kMaxRadix (sizes with prime factors above 5; its
// runtime-indexed arrays live in scratch, so only that kernel variant has it).
template <typename R>
__device__ void fft_stage_any(const Cx<R>* in, Cx<R>* out, const Cx<double>* __restrict__ W, int N, int B, int Ns,
                              int Rr, double sg) {
  const int M = N / Rr;
  const int stride = N / (Ns * Rr);
  for (int t = threadIdx.x; t < B * M; t += blockDim.x) {
    const int b = t / M, j = t - b * M, k = j % Ns;
    Cx<R> v[kMaxRadix];
    for (int r = 0; r < Rr; ++r) {
      Cx<R> x = in[b * N + j + r * M];
      if (r > 0 && k > 0) x = cmul(x, twiddle<R>(W, k * r * stride, sg));
      v[r] = x;
    }
    const int idxD = (j / Ns) * Ns * Rr + k;
    for (int m = 0; m < Rr; ++m) {
      double sx = 0.0, sy = 0.0;
      for (int r = 0; r < Rr; ++r) {
        const Cx<R> w = twiddle<R>(W, ((r * m) % Rr) * (N / Rr), sg);
        sx += (double)v[r].x * (double)w.x - (double)v[r].y * (double)w.y;
        sy += (double)v[r].x * (double)w.y + (double)v[r].y * (double)w.x;
      }
      out[b * N + idxD + m * Ns] = Cx<R>{(R)sx, (R)sy};
    }
  }
}

// Quotient and remainder by d; P2: d is a power of two (shift and mask
// instead of an integer division).
template <bool P2>
__device__ __forceinline__ int idiv(int x, int d) {
  if constexpr (P2) return x >> __builtin_ctz((unsigned)d);
  else return x / d;
}
template <bool P2>
__device__ __forceinline__ int imod(int x, int d) {
  if constexpr (P2) return x & (d - 1);
  else return x % d;
}

// LDS position of element x of line b in the single-buffer kernel: one
// complex of padding after every 16 and lines lane_stride(N) apart.  A 16-byte
// element per lane and 64 banks of 4 bytes make 16 slots per bank row; the
// Stockham writes of the first stages go out at strides of 4 and 16
// elements, which without the padding put 16 lanes on one slot.  The
// gathers of the strided axes take 8 lines at once: with gather = true the
// line stride is 4 slots (mod 16), which spreads them over the bank row (not
// in the binning pass, whose histogram would then push a block past a
// quarter of the CU's LDS).
__host__ __device__ constexpr int lane_stride(int N, bool gather = false) {
  return N + (N + 15) / 16 + (gather ? 4 : 0);
}
__device__ __forceinline__ int lpos(int b, int x, int LS) { return b * LS + x + (x >> 4); }

// In-place variant of a stage for the single-buffer kernel: every thread
// takes up to PMAX butterflies' inputs (twiddled) into registers, the block
// synchronises, then the outputs overwrite the same LDS lines.  The launch
// guarantees B N / RAD <= PMAX blockDim.x.  P2: N and B are powers of two.
template <typename R, int RAD, int PMAX, bool P2 = false>
__device__ __forceinline__ void fft_stage_inplace(Cx<R>* buf, const Cx<double>* Wl, int N, int B, int LS, int Ns,
                                                  double sg) {
  const int M = N / RAD;
  const int stride = N / (Ns * RAD);
  const int nbf = B * M;
  Cx<R> v[PMAX][RAD];
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    const int t = threadIdx.x + p * blockDim.x;
    if (t < nbf) {
      const int b = idiv<P2>(t, M), j = t - b * M, k = imod<P2>(j, Ns);
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        Cx<R> x = buf[lpos(b, j + r * M, LS)];
        if (r > 0 && k > 0) x = cmul(x, twiddle<R, true>(Wl, k * r * stride, sg));
        v[p][r] = x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    const int t = threadIdx.x + p * blockDim.x;
    if (t < nbf) {
      const int b = idiv<P2>(t, M), j = t - b * M, k = imod<P2>(j, Ns);
      Cx<R> o[RAD];
      small_dft<R, RAD, true>(v[p], o, Wl, N, sg);
      const int idxD = idiv<P2>(j, Ns) * Ns * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[lpos(b, idxD + r * Ns, LS)] = o[r];
    }
  }
  __syncthreads();
}

// Butterflies per thread the in-place stages hold in registers, by radix.
__host__ __device__ constexpr int inplace_pmax(int rad) { return rad == 2 ? 4 : rad == 3 ? 3 : rad == 8 ? 1 : 2; }

// radices the in-place kernel and the two-buffer kernel without the generic
// stage take (8: the binning pass's in-place kernel only)
__host__ __device__ constexpr bool fixed_radix(int rad) { return rad <= 5; }

// signed mode number of index i (Sec. 3.1: n~ in (-N/2, N/2])
__device__ __forceinline__ int wrapk(int i, int N) { return i <= N / 2 ? i : i - N; }

// shell floor(|n~|) of a mode with |n~|^2 = n2s (exact integer square root)
__device__ __forceinline__ int shell_of(int64_t n2s) {
  int b = (int)sqrt((double)n2s);
  while ((int64_t)(b + 1) * (b + 1) <= n2s) ++b;
  while ((int64_t)b * b > n2s) --b;
  return b;
}

// Input and output of a line pass: the plain pass reads and writes the
// complex array; the first (z) pass of a power spectrum reads the real field
// in storage precision instead, and its last (x) pass adds |f(n~)|^2 to
// per-block shell histograms instead of storing the transform.
enum LineMode { kLinePlain = 0, kLineRealIn = 1, kLineBinOut = 2 };
struct LineIO {
  const void* rin;  // kLineRealIn: the real field
  double* pS;       // kLineBinOut: nbins sums per block
  int nbins;
  int per_block;    // kLineBinOut: line batches per block
};

// Launch shape of the line passes, measured at 256^3 (a pass is held by the
// latency of its loads and LDS stages, not by HBM bandwidth):
// - a thread loads LU of its batch elements before it writes them to LDS:
//   two on the contiguous z lines (best of 1, 2, 4 and 8), one at a time on
//   the gathers of the strided axes, which got slower with more rows in
//   flight (1.0 : 1.06 : 1.25 for one, two and four);
// - at most 4 lines per z batch, so that more blocks share a CU (8 and 2
//   were slower);
// - up to 512 threads per block on the y pass (one butterfly per thread and
//   stage), 256 elsewhere.
// Radix-16 stages (two LDS round trips instead of four) and prefetching the
// next batch into registers were both slower: their register use halves the
// blocks per CU.
constexpr int kLineLoadsZ = 2;
constexpr int kLinesZ = 4;
constexpr int kThreadsY = 512;

// Sizes whose factors are all 2, 3, 4 or 5: one LDS buffer of B lines plus
// the N roots of unity, so that more blocks fit on a compute unit.
template <typename R, bool POW2, int MODE = kLinePlain, typename TIN = float, int LU = 1>
__global__ __launch_bounds__(512) void fft_lines_inplace_kernel(Cx<R>* data, const Cx<double>* __restrict__ W,
                                                                 FFTPlan P, int axis, int B, double sgn,
                                                                 double scale, LineIO io) {
  extern __shared__ unsigned char smem_raw[];
  const int N = P.N;
  Cx<double>* Wl = reinterpret_cast<Cx<double>*>(smem_raw);
  const int LS = lane_stride(N, axis != 2 && MODE != kLineBinOut);
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(Wl + lane_stride(N));  // the padded root table
  double* hist = reinterpret_cast<double*>(buf + (size_t)B * LS);  // kLineBinOut
  const size_t NN = (size_t)N * N;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int nzb = idiv<POW2>(N, B);
  // Blocks are dealt to the XCDs in turn; on the strided axes give each XCD
  // a contiguous range of batches instead, so that the row segments of
  // neighbouring batches (B elements each, under a cache line in FP32) are
  // fetched through one L2.
  int blk = blockIdx.x;
  if (axis != 2 && (gridDim.x & 7) == 0) blk = (blk & 7) * (gridDim.x >> 3) + (blk >> 3);
  int lb0 = blk, lb1 = blk + 1;
  if constexpr (MODE == kLineBinOut) {
    lb0 = blk * io.per_block;
    lb1 = min((int)(NN / B), lb0 + io.per_block);
    for (int h = tid; h < io.nbins; h += NT) hist[h] = 0.0;
  }
  for (int m = tid; m < N; m += NT) Wl[m + (m >> 4)] = W[m];
  for (int lb = lb0; lb < lb1; ++lb) {
    const int o = idiv<POW2>(lb, nzb), z0 = imod<POW2>(lb, nzb) * B;
    auto addr = [&](int b, int i) -> size_t {
      if (axis == 2) return ((size_t)lb * B + b) * N + i;
      if (axis == 1) return (size_t)o * NN + (size_t)i * N + z0 + b;
      return (size_t)i * NN + (size_t)o * N + z0 + b;
    };
    if (lb != lb0) __syncthreads();  // every thread is done with the previous batch
    // LU of a thread's elements are loaded before the first of them goes to LDS
    for (int e0 = tid; e0 < B * N; e0 += LU * NT) {
      Cx<R> in[LU];
#pragma unroll
      for (int k = 0; k < LU; ++k) {
        const int e = e0 + k * NT;
        if (e < B * N) {
          int b, i;
          if (axis == 2) { b = idiv<POW2>(e, N); i = imod<POW2>(e, N); } else { i = idiv<POW2>(e, B); b = imod<POW2>(e, B); }
          if constexpr (MODE == kLineRealIn)
            in[k] = Cx<R>{(R) static_cast<const TIN*>(io.rin)[addr(b, i)], R(0)};
          else
            in[k] = data[addr(b, i)];
        }
      }
#pragma unroll
      for (int k = 0; k < LU; ++k) {
        const int e = e0 + k * NT;
        if (e < B * N) {
          int b, i;
          if (axis == 2) { b = idiv<POW2>(e, N); i = imod<POW2>(e, N); } else { i = idiv<POW2>(e, B); b = imod<POW2>(e, B); }
          buf[lpos(b, i, LS)] = in[k];
        }
      }
    }
    __syncthreads();
    int Ns = 1;
    const double sg = sgn < 0.0 ? -1.0 : 1.0;
    for (int f = 0; f < P.nfac; ++f) {
      const int Rr = P.fac[f];
      // radix 8 (three stages instead of four at 256) is built into the
      // binning pass only, whose plan has it: its registers would cost the
      // other passes blocks per CU
      constexpr bool R8 = MODE == kLineBinOut;
      if (R8 && Rr == 8) {
        if constexpr (R8) fft_stage_inplace<R, 8, inplace_pmax(8), POW2>(buf, Wl, N, B, LS, Ns, sg);
      } else if constexpr (POW2) {  // power-of-two sizes: only radices 4 and 2 (fewer registers)
        if (Rr == 4) fft_stage_inplace<R, 4, inplace_pmax(4), true>(buf, Wl, N, B, LS, Ns, sg);
        else fft_stage_inplace<R, 2, inplace_pmax(2), true>(buf, Wl, N, B, LS, Ns, sg);
      } else {
        switch (Rr) {
          case 2: fft_stage_inplace<R, 2, inplace_pmax(2)>(buf, Wl, N, B, LS, Ns, sg); break;
          case 3: fft_stage_inplace<R, 3, inplace_pmax(3)>(buf, Wl, N, B, LS, Ns, sg); break;
          case 4: fft_stage_inplace<R, 4, inplace_pmax(4)>(buf, Wl, N, B, LS, Ns, sg); break;
          default: fft_stage_inplace<R, 5, inplace_pmax(5)>(buf, Wl, N, B, LS, Ns, sg); break;
        }
      }
      Ns *= Rr;
    }
    if constexpr (MODE == kLineBinOut) {
      // x pass, unscaled forward transform: mode (n1, n2, n3) = (x, line's y,
      // line's z).  Each thread takes a run of consecutive x on one line,
      // tracks the shell as n1 steps, and adds to the histogram once per
      // shell it meets rather than once per mode.
      const int tpl = NT / B, b = tid / tpl;
      if (b < B) {
        const int run = (N + tpl - 1) / tpl, i0 = (tid - b * tpl) * run, i1 = min(N, i0 + run);
        const int n2 = wrapk(o, N), n3 = wrapk(z0 + b, N);
        const int64_t r23 = (int64_t)n2 * n2 + (int64_t)n3 * n3;
        int sh = -1;
        double acc = 0.0;
        for (int i = i0; i < i1; ++i) {
          const int n1 = wrapk(i, N);
          const int64_t n2s = (int64_t)n1 * n1 + r23;
          int s2 = sh < 0 ? shell_of(n2s) : sh;
          while ((int64_t)(s2 + 1) * (s2 + 1) <= n2s) ++s2;
          while ((int64_t)s2 * s2 > n2s) --s2;
          if (s2 != sh) {
            if (sh >= 0) atomicAdd(&hist[sh], acc);
            sh = s2;
            acc = 0.0;
          }
          const Cx<R> v = buf[lpos(b, i, LS)];
          acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
        if (sh >= 0) atomicAdd(&hist[sh], acc);
      }
    } else {
      for (int e = tid; e < B * N; e += NT) {
        int b, i;
        if (axis == 2) { b = idiv<POW2>(e, N); i = imod<POW2>(e, N); } else { i = idiv<POW2>(e, B); b = imod<POW2>(e, B); }
        Cx<R> v = buf[lpos(b, i, LS)];
        v.x = (R)(v.x * scale);
        v.y = (R)(v.y * scale);
        data[addr(b, i)] = v;
      }
    }
  }
  if constexpr (MODE == kLineBinOut) {
    __syncthreads();
    for (int h = tid; h < io.nbins; h += NT) io.pS[(size_t)blockIdx.x * io.nbins + h] = hist[h];
  }
}

// One batch of B lines along `axis`, transformed with exponent sign `sgn`
// (+1: forward of Sec. 3.1, -1: inverse without the 1/N^3), then scaled.
// Lines along z are contiguous; along y and x a batch is B neighbouring z
// columns, so every row of the gather is B contiguous elements.
template <typename R, bool ANY>
__global__ __launch_bounds__(256) void fft_lines_kernel(Cx<R>* data, const Cx<double>* __restrict__ W, FFTPlan P,
                                                         int axis, int B, double sgn, double scale) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* bufA = reinterpret_cast<Cx<R>*>(smem_raw);
  Cx<R>* bufB = bufA + (size_t)B * P.N;
  const int N = P.N;
  const size_t NN = (size_t)N * N;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int lb = blockIdx.x;
  const int nzb = N / B;
  auto addr = [&](int b, int i) -> size_t {
    if (axis == 2) return ((size_t)lb * B + b) * N + i;
    const int o = lb / nzb, z0 = (lb % nzb) * B;
    if (axis == 1) return (size_t)o * NN + (size_t)i * N + z0 + b;
    return (size_t)i * NN + (size_t)o * N + z0 + b;
  };
  for (int e = tid; e < B * N; e += NT) {
    int b, i;
    if (axis == 2) { b = e / N; i = e % N; } else { i = e / B; b = e % B; }
    bufA[b * N + i] = data[addr(b, i)];
  }
  __syncthreads();
  Cx<R>* in = bufA;
  Cx<R>* out = bufB;
  int Ns = 1;
  const double sg = sgn < 0.0 ? -1.0 : 1.0;
  for (int f = 0; f < P.nfac; ++f) {
    const int Rr = P.fac[f];
    switch (Rr) {
      case 2: fft_stage<R, 2>(in, out, W, N, B, Ns, sg); break;
      case 3: fft_stage<R, 3>(in, out, W, N, B, Ns, sg); break;
      case 4: fft_stage<R, 4>(in, out, W, N, B, Ns, sg); break;
      case 5: fft_stage<R, 5>(in, out, W, N, B, Ns, sg); break;
      default:
        if constexpr (ANY) fft_stage_any<R>(in, out, W, N, B, Ns, Rr, sg);
        break;
    }
    __syncthreads();
    Cx<R>* tmp = in;
    in = out;
    out = tmp;
    Ns *= Rr;
  }
  for (int e = tid; e < B * N; e += NT) {
    int b, i;
    if (axis == 2) { b = e / N; i = e % N; } else { i = e / B; b = e % B; }
    Cx<R> v = in[b * N + i];
    v.x = (R)(v.x * scale);
    v.y = (R)(v.y * scale);
    data[addr(b, i)] = v;
  }
}

// Three line passes (z, y, x).  Lines per block B: the most that fit (one
// buffer of at most 2048 elements plus the roots for the in-place kernel,
// two buffers within 64 KiB for the generic one), at most kLinesZ along z,
// fewer where that leaves under 2048 blocks, but at least 8 on the strided
// axes so that each gathered row is 128 bytes.
template <typename R>
static int fft3d(Cx<R>* data, const Cx<double>* W, int N, double sgn, double scale, hipStream_t s) {
  const FFTPlan P = make_plan(N);
  bool any = false;
  for (int f = 0; f < P.nfac; ++f) {
    if (P.fac[f] > kMaxRadix) { set_error("FFT radix above 32"); return LAT_EINVAL; }
    any = any || !fixed_radix(P.fac[f]);
  }
  int Bmax = 32;
  if (any)
    while (Bmax > 1 && (size_t)2 * Bmax * N * sizeof(Cx<R>) > 65536) Bmax >>= 1;
  else
    while (Bmax > 1 && Bmax * N > 2048) Bmax >>= 1;
  while (Bmax > 1 && N % Bmax) Bmax >>= 1;
  for (int axis = 2; axis >= 0; --axis) {
    const int minB = axis == 2 ? 1 : std::min(Bmax, 8);
    int B = axis == 2 ? std::min(Bmax, kLinesZ) : Bmax;
    while (B > minB && (size_t)N * N / B < 2048) B >>= 1;
    const int nblk = (int)((size_t)N * N / B);
    // (the two-buffer kernel is built for 256 threads)
    const int nt = std::min(axis == 1 && !any ? kThreadsY : 256, std::max(64, (B * N / 4 + 63) / 64 * 64));
    const double sc = axis == 0 ? scale : 1.0;
    if (any) {
      const size_t shm = (size_t)2 * B * N * sizeof(Cx<R>);
      hipLaunchKernelGGL((fft_lines_kernel<R, true>), dim3(nblk), dim3(nt), shm, s, data, W, P, axis, B, sgn, sc);
    } else {
      for (int f = 0; f < P.nfac; ++f)
        if ((B * N / P.fac[f] + nt - 1) / nt > inplace_pmax(P.fac[f])) {
          set_error("FFT: in-place stage does not cover the batch");
          return LAT_EINVAL;
        }
      const size_t shm =
          (size_t)lane_stride(N) * sizeof(Cx<double>) + (size_t)B * lane_stride(N, axis != 2) * sizeof(Cx<R>);
      const bool p2 = (N & (N - 1)) == 0;
      if (axis == 2) {
        if (p2)
          hipLaunchKernelGGL((fft_lines_inplace_kernel<R, true, kLinePlain, float, kLineLoadsZ>), dim3(nblk), dim3(nt),
                             shm, s, data, W, P, axis, B, sgn, sc, LineIO{});
        else
          hipLaunchKernelGGL((fft_lines_inplace_kernel<R, false, kLinePlain, float, kLineLoadsZ>), dim3(nblk),
                             dim3(nt), shm, s, data, W, P, axis, B, sgn, sc, LineIO{});
      } else if (p2) {
        hipLaunchKernelGGL((fft_lines_inplace_kernel<R, true>), dim3(nblk), dim3(nt), shm, s, data, W, P, axis, B,
                           sgn, sc, LineIO{});
      } else {
        hipLaunchKernelGGL((fft_lines_inplace_kernel<R, false>), dim3(nblk), dim3(nt), shm, s, data, W, P, axis, B,
                           sgn, sc, LineIO{});
      }
    }
    CL_HIP(hipGetLastError());
  }
  return LAT_OK;
}

// Forward transform of a real field (stored as TIN) for its power spectrum,
// in precision R (FP64 roots; FP64 histograms): the z pass reads the field
// itself (no complex copy), the x pass bins |f(n~)|^2 into nblk per-block
// histograms pS (nbins each) instead of storing the transform.
// *nblk = 0 (nothing launched) where these passes do not apply: a radix
// above 5, or the x pass's buffer, roots and histogram above 64 KiB of LDS.
template <typename R, typename TIN = R>
static int fft3d_bins(const TIN* f, Cx<R>* data, const Cx<double>* W, int N, int nbins, double* pS,
                      int max_blocks, int* nblk, hipStream_t s) {
  *nblk = 0;
  const FFTPlan P = make_plan(N), P8 = make_plan(N, true);  // P8: the x (binning) pass
  for (int k = 0; k < P.nfac; ++k)
    if (!fixed_radix(P.fac[k])) return LAT_OK;
  int Bmax = 32;
  while (Bmax > 1 && Bmax * N > 2048) Bmax >>= 1;
  while (Bmax > 1 && N % Bmax) Bmax >>= 1;
  // lines per batch and threads per block of each pass, as in fft3d (an FP32
  // batch takes half the LDS of an FP64 one, so more blocks share a CU)
  int Bs[3], nts[3];
  for (int axis = 2; axis >= 0; --axis) {
    const int minB = axis == 2 ? 1 : std::min(Bmax, 8);
    int B = axis == 2 ? std::min(Bmax, kLinesZ) : Bmax;
    while (B > minB && (size_t)N * N / B < 2048) B >>= 1;
    Bs[axis] = B;
    nts[axis] = std::min(axis == 1 ? kThreadsY : 256, std::max(64, (B * N / 4 + 63) / 64 * 64));
    const FFTPlan& PL = axis == 0 ? P8 : P;
    for (int k = 0; k < PL.nfac; ++k)
      if ((B * N / PL.fac[k] + nts[axis] - 1) / nts[axis] > inplace_pmax(PL.fac[k])) {
        set_error("FFT: in-place stage does not cover the batch");
        return LAT_EINVAL;
      }
  }
  auto shm_of = [&](int axis) {
    return (size_t)lane_stride(N) * sizeof(Cx<double>) +
           (size_t)Bs[axis] * lane_stride(N, axis == 1) * sizeof(Cx<R>) +
           (axis == 0 ? (size_t)nbins * sizeof(double) : 0);
  };
  if (shm_of(0) > 65536) return LAT_OK;
  const int nbatch0 = (int)((size_t)N * N / Bs[0]);
  const int per = (nbatch0 + max_blocks - 1) / max_blocks;
  const int nb_bin = (nbatch0 + per - 1) / per;
  const LineIO io{f, pS, nbins, per};
  const bool pow2 = (N & (N - 1)) == 0;
#define CL_LINES(MODE, ...)                                                                                     \
  do {                                                                                                          \
    if (pow2)                                                                                                   \
      hipLaunchKernelGGL((fft_lines_inplace_kernel<R, true, MODE, ##__VA_ARGS__>), dim3(grid), dim3(nts[axis]), \
                         shm_of(axis), s, data, W, PL, axis, Bs[axis], 1.0, 1.0, io);                           \
    else                                                                                                        \
      hipLaunchKernelGGL((fft_lines_inplace_kernel<R, false, MODE, ##__VA_ARGS__>), dim3(grid),                  \
                         dim3(nts[axis]), shm_of(axis), s, data, W, PL, axis, Bs[axis], 1.0, 1.0, io);          \
  } while (0)
  for (int axis = 2; axis >= 0; --axis) {
    const int grid = axis == 0 ? nb_bin : (int)((size_t)N * N / Bs[axis]);
    const FFTPlan& PL = axis == 0 ? P8 : P;
    if (axis == 2) CL_LINES(kLineRealIn, TIN, kLineLoadsZ);
    else if (axis == 1) CL_LINES(kLinePlain);
    else CL_LINES(kLineBinOut);
    CL_HIP(hipGetLastError());
  }
#undef CL_LINES
  *nblk = nb_bin;
  return LAT_OK;
}

// ---------------------------------------------------------------------------
// spectrum
// ---------------------------------------------------------------------------
template <typename T, typename R>
__global__ void real_to_complex_kernel(const T* f, Cx<R>* c, int64_t V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < V) c[i] = Cx<R>{(R)f[i], (R)0};
}

// Per-block shell histograms of |f(n~)|^2 (FIELD) and, with GEOM, of the
// shell geometry (sum of |n~| and mode counts), which does not depend on the
// field.
template <typename R, bool GEOM, bool FIELD = true>
__global__ __launch_bounds__(256) void bin_kernel(const Cx<R>* F, int N, int nbins, int64_t per_block,
                                                  double* pS, double* pK, unsigned long long* pC) {
  extern __shared__ unsigned char smem_raw[];
  double* hS = reinterpret_cast<double*>(smem_raw);
  double* hK = hS + nbins;
  unsigned long long* hC = reinterpret_cast<unsigned long long*>(hK + nbins);
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    hS[b] = 0.0;
    if (GEOM) { hK[b] = 0.0; hC[b] = 0ull; }
  }
  __syncthreads();
  const int64_t V = (int64_t)N * N * N;
  const int64_t i0 = (int64_t)blockIdx.x * per_block;
  const int64_t i1 = min(V, i0 + per_block);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const int i3 = (int)(i % N), i2 = (int)((i / N) % N), i1x = (int)(i / ((int64_t)N * N));
    const int n1 = wrapk(i1x, N), n2 = wrapk(i2, N), n3 = wrapk(i3, N);
    const int64_t n2s = (int64_t)n1 * n1 + (int64_t)n2 * n2 + (int64_t)n3 * n3;
    const int b = shell_of(n2s);
    if (FIELD) {
      const Cx<R> v = F[i];
      atomicAdd(&hS[b], (double)v.x * (double)v.x + (double)v.y * (double)v.y);
    }
    if (GEOM) {
      atomicAdd(&hK[b], sqrt((double)n2s));
      atomicAdd(&hC[b], 1ull);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    pS[(size_t)blockIdx.x * nbins + b] = hS[b];
    if (GEOM) {
      pK[(size_t)blockIdx.x * nbins + b] = hK[b];
      pC[(size_t)blockIdx.x * nbins + b] = hC[b];
    }
  }
}

// Sum the per-block histograms in block order and normalise (Sec. 3.1):
//   k[b] = k_IR <|n~|>_shell,
//   delta[b] = (k_IR b)^3/(2 pi^2) (dx/N)^3 S_b / (4 pi b^2)   (b >= 1).
// One block per shell; each thread sums a strided subset of the per-block
// histograms in block order, then a fixed-shape tree in LDS (deterministic).
// Without GEOM, K and C keep the values of the first (GEOM) call.
template <bool GEOM>
__global__ __launch_bounds__(256) void bin_sum_kernel(const double* pS, const double* pK,
                                                      const unsigned long long* pC, int nblk, int nbins, double kIR,
                                                      double norm, double* S, double* K, double* D,
                                                      unsigned long long* C) {
  __shared__ double rs[256], rk[256];
  __shared__ unsigned long long rc[256];
  const int b = blockIdx.x, t = threadIdx.x;
  double s = 0.0, k = 0.0;
  unsigned long long c = 0;
  for (int j = t; j < nblk; j += 256) {
    s += pS[(size_t)j * nbins + b];
    if (GEOM) {
      k += pK[(size_t)j * nbins + b];
      c += pC[(size_t)j * nbins + b];
    }
  }
  rs[t] = s;
  rk[t] = k;
  rc[t] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      rs[t] += rs[t + w];
      rk[t] += rk[t + w];
      rc[t] += rc[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double pi = 3.14159265358979323846264338327950288;
    s = rs[0];
    S[b] = s;
    const double kb = kIR * (double)b;
    D[b] = b > 0 ? kb * kb * kb * norm * s / (4.0 * pi * (double)b * (double)b) : 0.0;
    if (GEOM) {
      c = rc[0];
      K[b] = c ? kIR * rk[0] / (double)c : 0.0;
      C[b] = c;
    }
  }
}

// ---------------------------------------------------------------------------
// initial conditions (Sec. 7.1)
// ---------------------------------------------------------------------------
struct ModeArgs {
  int N;
  int field;       // counter word 2
  uint64_t seed;
  double kIR, P0;  // P(k) = P0 / (2 a^2 w_k), P0 = (w*/f*)^2 (N/dx)^3
  double a, alpha, m2eff, Hhom, kcut;
  int deriv;       // 0: field modes, 1: derivative modes
};

// For every representative of {n~, -n~} (smaller linear index), draw two
// Rayleigh moduli and two uniform phases from Philox(counter = (lin, field,
// 0), key = seed) and form
//   df  = (|l| e^{i th_l} + |r| e^{i th_r}) / sqrt 2
//   df' = a^{-(1-alpha)} i w_k (|l| e^{i th_l} - |r| e^{i th_r}) / sqrt 2 - H df;
// the partner receives the complex conjugate.  Self-conjugate modes are 0.
__global__ void vacuum_modes_kernel(Cx<double>* F, ModeArgs M) {
  const int64_t V = (int64_t)M.N * M.N * M.N;
  const int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lin >= V) return;
  const int N = M.N;
  const int i3 = (int)(lin % N), i2 = (int)((lin / N) % N), i1 = (int)(lin / ((int64_t)N * N));
  const int j1 = (N - i1) % N, j2 = (N - i2) % N, j3 = (N - i3) % N;
  const int64_t par = ((int64_t)j1 * N + j2) * N + j3;
  if (lin > par) return;
  if (lin == par) { F[lin] = Cx<double>{0.0, 0.0}; return; }
  const int n1 = wrapk(i1, N), n2 = wrapk(i2, N), n3 = wrapk(i3, N);
  const double k = M.kIR * sqrt((double)n1 * n1 + (double)n2 * n2 + (double)n3 * n3);
  const double om2 = k * k + M.a * M.a * M.m2eff;
  if (!(om2 > 0.0) || (M.kcut > 0.0 && k > M.kcut)) {
    F[lin] = Cx<double>{0.0, 0.0};
    F[par] = Cx<double>{0.0, 0.0};
    return;
  }
  const double om = sqrt(om2);
  const double P = M.P0 / (2.0 * M.a * M.a * om);
  const Philox4 u = philox4x32_10((uint32_t)lin, (uint32_t)((uint64_t)lin >> 32), (uint32_t)M.field, 0u,
                                  (uint32_t)M.seed, (uint32_t)(M.seed >> 32));
  const double two32 = 4294967296.0, twopi = 6.283185307179586476925286766559;
  const double ul = ((double)u.v[0] + 0.5) / two32, ur = ((double)u.v[1] + 0.5) / two32;
  const double tl = twopi * ((double)u.v[2] + 0.5) / two32, tr = twopi * ((double)u.v[3] + 0.5) / two32;
  const double Rl = sqrt(-P * log(ul)), Rr = sqrt(-P * log(ur));
  double sl, cl, sr, cr;
  sincos(tl, &sl, &cl);
  sincos(tr, &sr, &cr);
  const double Lx = Rl * cl, Ly = Rl * sl, Rx = Rr * cr, Ry = Rr * sr;
  const double is2 = 0.70710678118654752440084436210485;
  Cx<double> v;
  if (!M.deriv) {
    v = Cx<double>{(Lx + Rx) * is2, (Ly + Ry) * is2};
  } else {
    const double c = pow(M.a, -(1.0 - M.alpha)) * om * is2;
    // i c (L - R) - H (L + R)/sqrt 2
    v = Cx<double>{-c * (Ly - Ry) - M.Hhom * (Lx + Rx) * is2, c * (Lx - Rx) - M.Hhom * (Ly + Ry) * is2};
  }
  F[lin] = v;
  F[par] = Cx<double>{v.x, -v.y};
}

// out = scale * (base + Re F / V) in storage precision
template <typename T>
__global__ void store_real_kernel(const Cx<double>* F, T* out, int64_t V, double base, double invV, double scale,
                                  int add_fluct) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const double v = base + (add_fluct ? F[i].x * invV : 0.0);
  out[i] = (T)(scale * v);
}

static double potential_host(const lattice_params& p, const double* phis) {
  const double a = phis[0], c = p.nf > 1 ? phis[1] : 0.0;
  if (is_u1(p)) {
    const double r2 = 0.5 * (a * a + c * c);  // |phi|^2 with phi = (phi0 + i phi1)/sqrt 2
    return p.lambda * r2 * r2 + p.m2[0] * r2;
  }
  double v = 0.5 * p.m2[0] * a * a + 0.25 * p.lambda * a * a * a * a;
  if (p.nf > 1) v += 0.5 * p.m2[1] * c * c + 0.5 * p.q * a * a * c * c;
  return v;
}

// d^2 V / d phi_f^2 at the homogeneous values
static double curvature_host(const lattice_params& p, int f) {
  const double a = p.phi0[0], c = p.nf > 1 ? p.phi0[1] : 0.0;
  if (is_u1(p)) {
    // V = lambda (phi0^2 + phi1^2)^2 / 4 + m2 (phi0^2 + phi1^2) / 2
    const double s = a * a + c * c, x = f == 0 ? a : c;
    return p.lambda * (s + 2.0 * x * x) + p.m2[0];
  }
  if (f == 0) return p.m2[0] + 3.0 * p.lambda * a * a + p.q * c * c;
  return p.m2[1] + p.q * a * a;
}

int run_fft3d(lattice* h, int sign, double scale) {
  Cx<double>* W = reinterpret_cast<Cx<double>*>(h->twiddle);
  if (!h->twiddle_ready) {
    hipLaunchKernelGGL(twiddle_kernel, dim3((h->p.N + 255) / 256), dim3(256), 0, h->stream, W, h->p.N);
    CL_HIP(hipGetLastError());
    h->twiddle_ready = true;
  }
  return fft3d(reinterpret_cast<Cx<double>*>(h->fft), W, h->p.N, (double)sign, scale, h->stream);
}

// Homogeneous values plus (optionally) vacuum fluctuations for the scalar
// model, then b from the Hubble constraint with the full-lattice energies.
int init_state(lattice* h) {
  const lattice_params& p = h->p;
  if (is_u1(p)) return u1_init_state(h);
  if (is_su2(p)) return su2_init_state(h);
  const int N = p.N;
  const int64_t V = (int64_t)N * N * N;
  const double a = p.a0, al = p.alpha;
  const bool fp32 = p.precision == LAT_FP32;
  const int nfield = p.nf;
  const double fmp2 = p.fstar_over_mp * p.fstar_over_mp;
  double rho_hom = 0.0;
  for (int f = 0; f < nfield; ++f) rho_hom += p.dphi0[f] * p.dphi0[f] / (2.0 * std::pow(a, 2.0 * al));
  rho_hom += potential_host(p, p.phi0);
  const double Hhom = p.expansion ? std::sqrt(fmp2 / 3.0 * std::pow(a, 2.0 * (al + 1.0)) * rho_hom) / a : 0.0;
  const int threads = 256;
  const int blocks = (int)((V + threads - 1) / threads);
  Cx<double>* F = reinterpret_cast<Cx<double>*>(h->fft);
  for (int f = 0; f < nfield; ++f) {
    for (int deriv = 0; deriv < 2; ++deriv) {
      const bool fluct = p.ic == LAT_IC_VACUUM;
      if (fluct) {
        ModeArgs M;
        M.N = N;
        M.field = f;
        M.seed = p.seed;
        M.kIR = p.kIR;
        M.P0 = p.omega_over_f * p.omega_over_f * std::pow((double)N / h->dx, 3.0);
        M.a = a;
        M.alpha = al;
        M.m2eff = curvature_host(p, f);
        M.Hhom = Hhom;
        M.kcut = p.kcut;
        M.deriv = deriv;
        hipLaunchKernelGGL(vacuum_modes_kernel, dim3(blocks), dim3(threads), 0, h->stream, F, M);
        CL_HIP(hipGetLastError());
        int rc = run_fft3d(h, -1, 1.0);
        if (rc) return rc;
      }
      const int comp = deriv ? nfield + f : f;
      const double base = deriv ? p.dphi0[f] : p.phi0[f];
      const double scale = deriv ? std::pow(a, 3.0 - al) : 1.0;  // pi = a^{3-alpha} phi'
      void* out = h->buf[h->cur][comp];
      if (fp32)
        hipLaunchKernelGGL(store_real_kernel<float>, dim3(blocks), dim3(threads), 0, h->stream, F, (float*)out, V,
                           base, 1.0 / (double)V, scale, fluct ? 1 : 0);
      else
        hipLaunchKernelGGL(store_real_kernel<double>, dim3(blocks), dim3(threads), 0, h->stream, F, (double*)out,
                           V, base, 1.0 / (double)V, scale, fluct ? 1 : 0);
      CL_HIP(hipGetLastError());
    }
  }
  int rc = upload_scalars(h, a, 0.0, 0.0);
  if (rc) return rc;
  h->staggered = 0;
  h->step = 0;
  if (p.expansion) {
    rc = (is_u1(p)) ? u1_energies(h) : scalar_energies(h);
    if (rc) return rc;
    DevState d;
    CL_HIP(hipMemcpyAsync(&d, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    CL_HIP(hipStreamSynchronize(h->stream));
    const double b0 = std::sqrt(fmp2 / 3.0 * std::pow(a, 2.0 * (al + 1.0)) * d.obs.rho);
    rc = upload_scalars(h, a, b0, 0.0);
    if (rc) return rc;
  }
  return LAT_OK;
}

}  // namespace cl

using namespace cl;

namespace {

// FFT of one component and its shell histogram, left on the device:
// S (sum |f|^2), K (mean k), D (delta with 4 pi b^2), C (counts), nb shells.
struct Bins {
  double *S, *K, *D;
  unsigned long long* C;
  int nb;
};

// Shell sums of several real fields added (acc = sum_c f_c S_c, with
// f_c = a^pw read from the device state, or 1 for pw = 0), and the paper's
// delta of the sum.
__global__ void shell_accumulate_kernel(const double* S, double* acc, int nb, int first, const DevState* st,
                                        double pw) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double f = pw == 0.0 ? 1.0 : pow(st->a, pw);
  acc[b] = (first ? 0.0 : acc[b]) + f * S[b];
}

__global__ void shell_delta_kernel(const double* acc, double* D, int nb, double kIR, double norm) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double kb = kIR * (double)b;
  D[b] = b > 0 ? kb * kb * kb * norm * acc[b] / (4.0 * M_PI * (double)b * (double)b) : 0.0;
}

int component_bins(lattice_t* h, const void* src, Bins* out);

int spectrum_bins(lattice_t* h, int which, Bins* out) {
  const int N = h->p.N;
  const int nb = (int)std::floor(std::sqrt(3.0) * N / 2.0) + 1;
  int comp = -1;
  if (h->p.model == LAT_MODEL_SCALAR) {
    if (which >= 0 && which < h->p.nf) comp = which;
    else if (which >= 16 && which < 16 + h->p.nf) comp = h->p.nf + which - 16;
  } else if (is_su2(h->p)) {
    // the four real components of Phi and pi, or (Sec. 6.3.2) their sums
    if (which >= 0 && which < 4) comp = which;
    else if (which >= 16 && which < 20) comp = 4 + which - 16;
    else if (which == LAT_SPEC_U1_PHI || which == LAT_SPEC_U1_PI) {
      char* tail = h->spec + (size_t)(spec_blocks(N)) * nb * 24 + (size_t)nb * 32;
      double* acc = reinterpret_cast<double*>(tail);
      double* dacc = acc + nb;
      Bins B{};
      for (int c = 0; c < 4; ++c) {
        int rc = component_bins(h, h->buf[h->cur][(which == LAT_SPEC_U1_PHI ? 0 : 4) + c], &B);
        if (rc) return rc;
        hipLaunchKernelGGL(shell_accumulate_kernel, dim3((nb + 255) / 256), dim3(256), 0, h->stream, B.S, acc, nb,
                           c == 0 ? 1 : 0, h->st, 0.0);
        CL_HIP(hipGetLastError());
      }
      const double norm = std::pow(h->dx / N, 3.0) / (2.0 * M_PI * M_PI);
      hipLaunchKernelGGL(shell_delta_kernel, dim3((nb + 255) / 256), dim3(256), 0, h->stream, acc, dacc, nb,
                         h->p.kIR, norm);
      CL_HIP(hipGetLastError());
      *out = Bins{acc, B.K, dacc, B.C, nb};
      return LAT_OK;
    }
  } else {
    if (which >= 0 && which < 2) comp = which;                 // Re, Im of phi
    else if (which >= 16 && which < 18) comp = 2 + which - 16;  // Re, Im of pi
    else if (which >= LAT_SPEC_U1_PHI && which <= LAT_SPEC_U1_B) {
      // sums over components (Sec. 5.4.2): the complex scalar, its momentum,
      // E_i = pi_A,i / a^{1-alpha}, and B_i (computed into the free state buffer)
      const int nc = which <= LAT_SPEC_U1_PI ? 2 : 3;
      const double pw = which == LAT_SPEC_U1_E ? -2.0 * (1.0 - h->p.alpha) : 0.0;
      char* tail = h->spec + (size_t)(spec_blocks(N)) * nb * 24 + (size_t)nb * 32;
      double* acc = reinterpret_cast<double*>(tail);
      double* dacc = acc + nb;
      Bins B{};
      for (int c = 0; c < nc; ++c) {
        const void* src;
        if (which == LAT_SPEC_U1_PHI) src = h->buf[h->cur][c];
        else if (which == LAT_SPEC_U1_PI) src = h->buf[h->cur][2 + c];
        else if (which == LAT_SPEC_U1_E) src = h->buf[h->cur][7 + c];
        else {
          void* scratch = h->buf[1 - h->cur][0];
          int rc = u1_magnetic_field(h, c, scratch);
          if (rc) return rc;
          src = scratch;
        }
        int rc = component_bins(h, src, &B);
        if (rc) return rc;
        hipLaunchKernelGGL(shell_accumulate_kernel, dim3((nb + 255) / 256), dim3(256), 0, h->stream, B.S, acc, nb,
                           c == 0 ? 1 : 0, h->st, pw);
        CL_HIP(hipGetLastError());
      }
      const double norm = std::pow(h->dx / N, 3.0) / (2.0 * M_PI * M_PI);
      hipLaunchKernelGGL(shell_delta_kernel, dim3((nb + 255) / 256), dim3(256), 0, h->stream, acc, dacc, nb,
                         h->p.kIR, norm);
      CL_HIP(hipGetLastError());
      *out = Bins{acc, B.K, dacc, B.C, nb};
      return LAT_OK;
    }
  }
  if (comp < 0) { set_error("spectrum: unknown field selector"); return LAT_EINVAL; }
  return component_bins(h, h->buf[h->cur][comp], out);
}

int component_bins(lattice_t* h, const void* src, Bins* out) {
  const int N = h->p.N;
  const int nb = (int)std::floor(std::sqrt(3.0) * N / 2.0) + 1;
  const int64_t V = (int64_t)N * N * N;
  const int threads = 256;
  const int blocks = (int)((V + threads - 1) / threads);
  Cx<double>* F = reinterpret_cast<Cx<double>*>(h->fft);
  const int nblk = spec_blocks(N);
  const int64_t per = (V + nblk - 1) / nblk;
  double* pS = (double*)h->spec;
  double* pK = pS + (size_t)nblk * nb;
  unsigned long long* pC = (unsigned long long*)(pK + (size_t)nblk * nb);
  double* S = (double*)(pC + (size_t)nblk * nb);
  double* K = S + nb;
  double* D = K + nb;
  unsigned long long* C = (unsigned long long*)(D + nb);
  const size_t shm = (size_t)nb * 24;
  const double norm = std::pow(h->dx / N, 3.0) / (2.0 * M_PI * M_PI);
  // Sizes with radices up to 5: the transform reads the field and bins its
  // last pass itself; the shell geometry (K, C) is binned once, from the mode
  // indices alone, and found in place by later calls (nothing else writes it).
  Cx<double>* W = reinterpret_cast<Cx<double>*>(h->twiddle);
  if (!h->twiddle_ready) {
    hipLaunchKernelGGL(twiddle_kernel, dim3((N + 255) / 256), dim3(256), 0, h->stream, W, N);
    CL_HIP(hipGetLastError());
    h->twiddle_ready = true;
  }
  int fused_blk = 0;
  if (!h->spec_geom_ready) {
    // geometry only (no field reads); S is overwritten below
    hipLaunchKernelGGL((bin_kernel<double, true, false>), dim3(nblk), dim3(256), shm, h->stream, F, N, nb, per, pS,
                       pK, pC);
    CL_HIP(hipGetLastError());
    hipLaunchKernelGGL(bin_sum_kernel<true>, dim3(nb), dim3(256), 0, h->stream, pS, pK, pC, nblk, nb, h->p.kIR,
                       norm, S, K, D, C);
    CL_HIP(hipGetLastError());
    h->spec_geom_ready = true;
  }
  // The transform runs in FP64 for either storage: an FP32 transform's
  // rounding is relative to the field's total power (the zero mode of a
  // condensate included), which would swamp the low-power shells.
  int rc = h->p.precision == LAT_FP32
               ? fft3d_bins<double, float>((const float*)src, F, W, N, nb, pS, nblk, &fused_blk, h->stream)
               : fft3d_bins<double, double>((const double*)src, F, W, N, nb, pS, nblk, &fused_blk, h->stream);
  if (rc) return rc;
  if (fused_blk > 0) {
    hipLaunchKernelGGL(bin_sum_kernel<false>, dim3(nb), dim3(256), 0, h->stream, pS, pK, pC, fused_blk, nb,
                       h->p.kIR, norm, S, K, D, C);
    CL_HIP(hipGetLastError());
    *out = Bins{S, K, D, C, nb};
    return LAT_OK;
  }
  // other sizes: complex copy, the general transform, then the binning kernel
  if (h->p.precision == LAT_FP32)
    hipLaunchKernelGGL((real_to_complex_kernel<float, double>), dim3(blocks), dim3(threads), 0, h->stream,
                       (const float*)src, F, V);
  else
    hipLaunchKernelGGL((real_to_complex_kernel<double, double>), dim3(blocks), dim3(threads), 0, h->stream,
                       (const double*)src, F, V);
  CL_HIP(hipGetLastError());
  rc = run_fft3d(h, +1, 1.0);
  if (rc) return rc;
  hipLaunchKernelGGL((bin_kernel<double, false>), dim3(nblk), dim3(256), shm, h->stream, F, N, nb, per, pS, pK, pC);
  CL_HIP(hipGetLastError());
  hipLaunchKernelGGL(bin_sum_kernel<false>, dim3(nb), dim3(256), 0, h->stream, pS, pK, pC, nblk, nb, h->p.kIR,
                     norm, S, K, D, C);
  CL_HIP(hipGetLastError());
  *out = Bins{S, K, D, C, nb};
  return LAT_OK;
}

// log10 of the mode-averaged spectrum kbar^3 norm S_b / C_b at nk log-spaced
// k from kIR to kIR (nb - 1), linear in log k between the centres of shells
// b >= 1 with modes and positive power, constant beyond the end shells.
// One block: the usable shells are compacted in order into LDS (their
// centres increase with b), then each output finds its bracket by bisection.
constexpr int kLogkMaxBins = 1024;
__global__ __launch_bounds__(1024) void logk_kernel(const double* S, const double* K, const unsigned long long* C,
                                                    int nb, double norm, double kIR, int nk, float* out) {
  __shared__ double xs[kLogkMaxBins], ys[kLogkMaxBins];
  __shared__ int pos[kLogkMaxBins];
  const int t = threadIdx.x;
  const bool ok = t >= 1 && t < nb && C[t] != 0ull && S[t] > 0.0;
  pos[t] = ok ? 1 : 0;
  __syncthreads();
  for (int w = 1; w < kLogkMaxBins; w <<= 1) {  // inclusive prefix sum of the flags
    const int v = t >= w ? pos[t - w] : 0;
    __syncthreads();
    pos[t] += v;
    __syncthreads();
  }
  const int nv = pos[kLogkMaxBins - 1];
  if (ok) {
    const double kb = K[t];
    xs[pos[t] - 1] = log10(kb);
    ys[pos[t] - 1] = log10(kb * kb * kb * norm * S[t] / (double)C[t]);
  }
  __syncthreads();
  const double lo = log10(kIR), hi = log10(kIR * (double)(nb - 1));
  for (int j = t; j < nk; j += blockDim.x) {
    const double x = lo + (hi - lo) * (double)j / (double)(nk - 1);
    double res;
    if (nv == 0) {
      res = -INFINITY;
    } else {
      int a = 0, e = nv;  // first i with x <= xs[i]
      while (a < e) {
        const int m = (a + e) >> 1;
        if (x <= xs[m]) e = m; else a = m + 1;
      }
      if (a == 0) res = ys[0];
      else if (a == nv) res = ys[nv - 1];
      else res = ys[a - 1] + (x - xs[a - 1]) / (xs[a] - xs[a - 1]) * (ys[a] - ys[a - 1]);
    }
    out[j] = (float)res;
  }
}

}  // namespace

extern "C" int lattice_spectrum(lattice_t* h, int which, int nbins_cap, double* k, double* delta, double* sum_sq,
                                int64_t* counts, int* nbins) {
  if (!h || !k || !delta || !sum_sq || !counts || !nbins) { set_error("NULL argument"); return LAT_EINVAL; }
  const int nb = (int)std::floor(std::sqrt(3.0) * h->p.N / 2.0) + 1;
  *nbins = nb;
  if (nbins_cap < nb) { set_error("nbins_cap too small: need " + std::to_string(nb)); return LAT_ENOMEM; }
  Bins B;
  int rc = spectrum_bins(h, which, &B);
  if (rc) return rc;
  std::vector<unsigned long long> hC(nb);
  CL_HIP(hipMemcpyAsync(sum_sq, B.S, nb * 8, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipMemcpyAsync(k, B.K, nb * 8, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipMemcpyAsync(delta, B.D, nb * 8, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipMemcpyAsync(hC.data(), B.C, nb * 8, hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipStreamSynchronize(h->stream));
  for (int b = 0; b < nb; ++b) counts[b] = (int64_t)hC[b];
  return LAT_OK;
}

extern "C" int lattice_spectrum_logk(lattice_t* h, int which, int nk, float* dev_out) {
  if (!h || !dev_out) { set_error("NULL argument"); return LAT_EINVAL; }
  if (nk < 2 || nk > 4096) { set_error("nk must be in [2, 4096]"); return LAT_EINVAL; }
  Bins B;
  int rc = spectrum_bins(h, which, &B);
  if (rc) return rc;
  const double norm = std::pow(h->dx / h->p.N, 3.0) / (2.0 * M_PI * M_PI);
  if (B.nb > kLogkMaxBins) { set_error("spectrum_logk: too many shells"); return LAT_EINVAL; }
  hipLaunchKernelGGL(logk_kernel, dim3(1), dim3(kLogkMaxBins), 0, h->stream, B.S, B.K, B.C, B.nb, norm,
                     h->p.kIR, nk, dev_out);
  CL_HIP(hipGetLastError());
  return LAT_OK;
}
