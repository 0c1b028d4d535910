// Complex scalar with compact U(1) links on gfx950 (Sec. 5.3: staggered
// leapfrog, velocity Verlet and its Yoshida compositions).  Every pass is the
// drift of one (sub-)step followed by the merged kicks that close it and open
// the next, read from one state buffer and written to the other, then an
// FP64 finish that advances a and b; the pass sequence is the scalar path's.
//
// Components (storage precision, N^3 each): 0,1 = Re, Im phi; 2,3 = Re, Im
// pi; 4 + i = phase th_i of the link V_i = exp(i th_i); 7 + i = piA_i.
// A compact U(1) link is a point on the unit circle, so its phase is an exact
// coordinate: plaquettes are V_ij = exp(i Phi_ij) with
// Phi_ij(n) = th_i(n) + th_j(n+i) - th_i(n+j) - th_j(n), 1 - Re V_ij =
// 2 sin^2(Phi_ij/2) without cancellation, and |V| = 1 holds exactly in FP32.
//
// Kernels (Sec. 5.1, 5.3):
//   K_phi   = -a^{3+alpha}(2 lambda |phi|^2 + m2) phi
//             + a^{1+alpha} sum_i (V_i phi_{+i} - 2 phi + conj V_i(n-i) phi_{-i}) / dx^2
//   K_{A,i} = a^{1+alpha}(2 e/dx)(f/w)^2 Im[conj phi V_i phi_{+i}]
//             + a^{alpha-1}/(e dx^3) sum_{j!=i} (Im V_ij(n) - Im V_ij(n-j)),
//   V_ij(n) = V_i(n) V_j(n+i) conj V_i(n+j) conj V_j(n).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"
#include "internal.hpp"
#include "phase.hpp"

namespace cl {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};
template <typename T>
__device__ __forceinline__ C2<T> cm(C2<T> a, C2<T> b) {
  return C2<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cc(C2<T> a) {
  return C2<T>{a.x, -a.y};
}

// arguments of the Gauss-law residual kernel
template <typename T>
struct U1Args {
  T* c[10];
  int N;
  double dx, alpha, fmp2, lam, m2, e, wf2, h;
  int expand;
  double* partials;
  DevState* st;
};

constexpr int kU1Acc = 11;
// the workspace reserves 16 FP64 partials per 256-site block
static_assert(kU1Acc <= 16, "U(1) partials exceed the reserved region");

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-block sums of NT threads' accumulators (waves in order) into the
// block's record.
template <int NT, int NACC>
__device__ void u1_block_partials(double (&acc)[NACC], double* partials) {
  constexpr int NW = NT / 64;
  __shared__ double red[NW][NACC];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    const double s = wsum(acc[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (tid < NACC) {
    double s = red[0][tid];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += red[w][tid];
    partials[(size_t)blockIdx.x * NACC + tid] = s;
  }
}

template <typename T>
__device__ __forceinline__ C2<T> ld(const T* re, const T* im, size_t i) {
  return C2<T>{re[i], im[i]};
}

// Gauss residual G(n) = sum_i (piA_i(n) - piA_i(n-i))/dx - 2e (f/w)^2 Im[conj phi pi]
template <typename T>
__global__ __launch_bounds__(256) void u1_gauss_kernel(U1Args<T> A) {
  const int N = A.N;
  const size_t NN = (size_t)N * N;
  const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int x = (int)(s / NN), y = (int)((s / N) % N), z = (int)(s % N);
  const size_t sm[3] = {(size_t)((x - 1 + N) % N) * NN + (size_t)y * N + z,
                        (size_t)x * NN + (size_t)((y - 1 + N) % N) * N + z,
                        (size_t)x * NN + (size_t)y * N + (z - 1 + N) % N};
  double div = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) div += ((double)A.c[7 + i][s] - (double)A.c[7 + i][sm[i]]) / A.dx;
  const double rho = 2.0 * A.e / A.wf2 *
                     ((double)A.c[0][s] * (double)A.c[3][s] - (double)A.c[1][s] * (double)A.c[2][s]);
  double acc[4] = {(div - rho) * (div - rho), div * div, rho * rho, rho};
  u1_block_partials<256>(acc, A.partials);
}

__global__ __launch_bounds__(1024) void u1_gauss_finish_kernel(const double* partials, int nblocks, DevState* st) {
  __shared__ double red[16][4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < nblocks; b += 1024)
    for (int k = 0; k < 4; ++k) tot[k] += partials[(size_t)b * 4 + k];
  for (int k = 0; k < 4; ++k) {
    const double s = wsum(tot[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (tid != 0) return;
  double S[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; ++k)
    for (int w = 0; w < 16; ++w) S[k] += red[w][k];
  const double den = sqrt(S[1]) + sqrt(S[2]);
  st->obs.gauss = den > 0.0 ? sqrt(S[0]) / den : 0.0;
}

// ---------------------------------------------------------------------------
// The pass kernel.  A block owns a TY x TZ tile of the (y, z) plane and marches along x over XC
// planes.  Each plane enters LDS already drifted (phi and the link phases,
// with a one-site ring including corners, the ring drifted redundantly); two
// planes are held, x and x+1.  Per plane the block first computes the
// plaquette sines S_01, S_02, S_12 of its sites and of the y-1 row and z-1
// column, shared through LDS, so that every plaquette sine is evaluated once
// instead of once per use.  Values of plane x-1 that the kick needs (phi,
// theta_0, S_01, S_02 of the own column) stay in registers.
// ---------------------------------------------------------------------------
// One pass (as PassDesc of the scalar path, Sec. 3.3.2 merged kicks):
//   a'  = a + wd h b,  a_mid = (a + a')/2
//   phi = phi + wd h pi / a_mid^{3-alpha},  V = Cayley(wd h, piA, a_mid) V
//   pi  = pi + (wk1 + wk2) h K_phi(a'),     piA = piA + (wk1 + wk2) h K_A(a')
// E_K from pi_in and pi + wk1 h K (VV) or from the mean of <pi_in^2> and
// <pi_out^2> (LF), likewise for piA.
template <typename T>
struct U1PassArgs {
  const T* src[10];
  T* dst[10];
  int N, XC, swizzle;
  double dx, alpha, fmp2, lam, m2, e, wf2, h;
  int expand;
  PassDesc pd;
  double* partials;
  DevState* st;
  PrevPass prev;  // finish of the previous pass of a chain (partials == nullptr: none)
};

template <typename T>
__device__ void u1_finish_state(const U1PassArgs<T>& A, const PassDesc& pd, const DevState* in,
                                const double (&S)[kU1Acc], DevState* out, double& a_next, double& b_next);
template <int NT>
__device__ bool u1_reduce_partials(const double* partials, int nb, double (&S)[kU1Acc]);

template <typename T>
__device__ __forceinline__ T wrap_phase(T t) {
  // any integer count of turns gives the same link, so the turn count may
  // come from a product with 1/(2 pi)
  const T twopi = (T)6.283185307179586476925286766559;
  return t - twopi * rint(t * (T)0.15915494309189533576888376337251);
}

// NC: non-compact gauge field (Sec. 5.2).  The three link slots then hold A_i;
// the drift is linear, the link phase is theta_i = -e dx A_i, and the
// plaquette terms are the angles themselves (Phi = -e dx^2 F_ij; Phi^2/2 for
// the magnetic energy), which turns the compact kernels into the quadratic
// ones with the same coefficients.
template <typename T, int TZ, int BY, int RY, bool NC>
__global__ __launch_bounds__(TZ* BY) void u1_pass_kernel(U1PassArgs<T> A) {
  constexpr int TY = BY * RY, NT = TZ * BY, LY = TY + 2, LZ = TZ + 2;
  constexpr int NH = 2 * LZ + 2 * TY;  // ring of the (TY+2) x (TZ+2) plane tile
  static_assert(NH <= NT, "ring larger than block");
  static_assert(TZ + TY <= NT, "low ring larger than block");
  static_assert(NT == 256, "partials and LDS sized for four waves");
  __shared__ T Lp[2][2][LY][LZ];       // drifted phi (Re, Im), planes in flight
  __shared__ T Lt[2][3][LY][LZ];       // drifted link phases (own sites are stored)
  __shared__ C2<T> Lu[2][3][LY][LZ];   // drifted links minus one, U_i - 1 = (cos - 1, sin)
  __shared__ T Ls[3][TY + 1][TZ + 1];  // S_01, S_02, S_12; index 0 = row y0-1 / column z0-1

  const int N = A.N;
  const int NN = N * N;
  const int tid = threadIdx.x, tz = tid % TZ, ty = tid / TZ;
  int bid = blockIdx.x;
  if (A.swizzle) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  const int nzt = N / TZ, nyt = N / TY;
  const int z0 = (bid % nzt) * TZ;
  const int y0 = ((bid / nzt) % nyt) * TY;
  const int x0 = (bid / (nzt * nyt)) * A.XC;

  // ring site owned by this thread (one at most)
  const bool has_ring = tid < NH;
  int rly = 0, rlz = 0;
  if (tid < LZ) { rly = 0; rlz = tid; }
  else if (tid < 2 * LZ) { rly = TY + 1; rlz = tid - LZ; }
  else if (tid < 2 * LZ + TY) { rly = 1 + tid - 2 * LZ; rlz = 0; }
  else { rly = 1 + tid - 2 * LZ - TY; rlz = TZ + 1; }
  const int ry_g = (y0 - 1 + rly + N) % N, rz_g = (z0 - 1 + rlz + N) % N;
  // low-ring site whose plaquette sines this thread computes (row y0-1 or column z0-1)
  const bool has_low = tid < TZ + TY;
  const int sly = tid < TZ ? 0 : 1 + tid - TZ;
  const int slz = tid < TZ ? 1 + tid : 0;

  auto site = [&](int x, int y, int z) -> int { return x * NN + y * N + z; };

  // raw values: own column (RY rows) and the ring site of plane x
  T raw[10][RY], rraw[10];
  auto load_plane = [&](int x) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int o = site(x, y0 + r * BY + ty, z0 + tz);
#pragma unroll
      for (int c = 0; c < 10; ++c) raw[c][r] = A.src[c][o];
    }
    if (has_ring) {
      const int o = site(x, ry_g, rz_g);
#pragma unroll
      for (int c = 0; c < 10; ++c) rraw[c] = A.src[c][o];
    }
  };
  // plane x0-1 is loaded before the previous pass's finish is applied (the
  // loads need no coefficients), so that their latency overlaps it
  load_plane((x0 - 1 + N) % N);

  // homogeneous coefficients (FP64, the same in every block); a chained pass
  // first applies the previous pass's finish (every block, same order)
  double a_in, b_in;
  if (A.prev.partials) {
    __shared__ double ab[2];
    double S[kU1Acc];
    if (u1_reduce_partials<NT>(A.prev.partials, A.prev.nblocks, S)) {
      double an, bn;
      u1_finish_state<T>(A, A.prev.pd, A.st, S, blockIdx.x == 0 ? A.prev.out : nullptr, an, bn);
      ab[0] = an;
      ab[1] = bn;
    }
    __syncthreads();
    a_in = ab[0];
    b_in = ab[1];
  } else {
    a_in = A.st->a;
    b_in = A.st->b;
  }
  const double anew = A.expand ? a_in + A.pd.wd * A.h * b_in : a_in;
  const double amid = 0.5 * (a_in + anew);
  const bool dr = A.pd.wd != 0.0;
  const double hw = A.pd.wd * A.h;
  // per-pass coefficients as hi + lo pairs (no coherent rounding of them)
  const Coef<T> cd = ucoef<T>(dr ? hw * apow(amid, -(3.0 - A.alpha)) : 0.0);
  const Coef<T> cu = ucoef<T>(dr ? A.e * hw * A.dx / (2.0 * apow(amid, 1.0 - A.alpha)) : 0.0);
  const Coef<T> cA = ucoef<T>(dr ? hw / apow(amid, 1.0 - A.alpha) : 0.0);  // non-compact A drift
  const Coef<T> mth = ucoef<T>(-A.e * A.dx);                                // theta = -e dx A
  const Coef<T> cl = ucoef<T>(apow(anew, 1.0 + A.alpha) / (A.dx * A.dx));
  const Coef<T> cp = ucoef<T>(apow(anew, 3.0 + A.alpha));
  const Coef<T> cj = ucoef<T>(apow(anew, 1.0 + A.alpha) * 2.0 * A.e / A.dx / A.wf2);
  const Coef<T> cb = ucoef<T>(apow(anew, A.alpha - 1.0) / (A.e * A.dx * A.dx * A.dx));
  const Coef<T> ck = ucoef<T>((A.pd.wk1 + A.pd.wk2) * A.h);
  const Coef<T> cE = ucoef<T>((A.pd.mode == MODE_LF ? A.pd.wk1 + A.pd.wk2 : A.pd.wk1) * A.h);
  const bool wr = A.pd.write != 0;
  const T lam = (T)A.lam, m2 = (T)A.m2;
  const Coef<T> lam2c = ucoef<T>(2.0 * A.lam), m2c = ucoef<T>(A.m2);

  // drift the raw values into LDS buffer b
  // (the only transcendentals of the pass: one arctangent and one sincos per link)
  auto drift_into = [&](int b) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ly = 1 + r * BY + ty, lz = 1 + tz;
      Lp[b][0][ly][lz] = fma_c(cd, raw[2][r], raw[0][r]);
      Lp[b][1][ly][lz] = fma_c(cd, raw[3][r], raw[1][r]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T th;
        if constexpr (NC) {
          th = fma_c(cA, raw[7 + i][r], raw[4 + i][r]);  // A_i after the drift
        } else {
          th = dr ? wrap_phase(raw[4 + i][r] - T(2) * atan_t(mul_c(cu, raw[7 + i][r]))) : raw[4 + i][r];
        }
        Lt[b][i][ly][lz] = th;
        T sn, cm;
        sincos_m1(NC ? mul_c(mth, th) : th, &sn, &cm);
        Lu[b][i][ly][lz] = C2<T>{cm, sn};
      }
    }
    if (has_ring) {
      Lp[b][0][rly][rlz] = fma_c(cd, rraw[2], rraw[0]);
      Lp[b][1][rly][rlz] = fma_c(cd, rraw[3], rraw[1]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T th;
        if constexpr (NC) {
          th = fma_c(cA, rraw[7 + i], rraw[4 + i]);
          Lt[b][i][rly][rlz] = th;  // the plaquette angles need A on the ring
        } else {
          th = dr ? wrap_phase(rraw[4 + i] - T(2) * atan_t(mul_c(cu, rraw[7 + i]))) : rraw[4 + i];
        }
        T sn, cm;
        sincos_m1(NC ? mul_c(mth, th) : th, &sn, &cm);
        Lu[b][i][rly][rlz] = C2<T>{cm, sn};
      }
    }
  };
  // plaquettes of site (ly, lz) of plane buffer c (plane x+1 in buffer n) as
  // products of links, P_ij(m) = U_i(m) U_j(m+i) U_i(m+j)^* U_j(m)^* = e^{i Phi_ij}:
  // sin Phi_ij = Im P and 1 - cos Phi_ij = (Im P)^2 / (1 + Re P) (no cancellation
  // for small Phi; 1 - Re P where Re P < 0).
  auto plaq = [&](int c, int n, int ly, int lz, T (&sn)[3], T (&om)[3]) {
    if constexpr (NC) {
      // Phi_ij = theta_i(m) + theta_j(m+i) - theta_i(m+j) - theta_j(m) with theta = -e dx A
      const T a0 = Lt[c][0][ly][lz], a1 = Lt[c][1][ly][lz], a2 = Lt[c][2][ly][lz];
      sn[0] = mul_c(mth, (a0 + Lt[n][1][ly][lz]) - (Lt[c][0][ly + 1][lz] + a1));
      sn[1] = mul_c(mth, (a0 + Lt[n][2][ly][lz]) - (Lt[c][0][ly][lz + 1] + a2));
      sn[2] = mul_c(mth, (a1 + Lt[c][2][ly + 1][lz]) - (Lt[c][1][ly][lz + 1] + a2));
#pragma unroll
      for (int k = 0; k < 3; ++k) om[k] = T(0.5) * sn[k] * sn[k];
      return;
    }
    auto U = [](C2<T> m) { return C2<T>{T(1) + m.x, m.y}; };
    const C2<T> u0 = U(Lu[c][0][ly][lz]), u1 = U(Lu[c][1][ly][lz]), u2 = U(Lu[c][2][ly][lz]);
    C2<T> P[3];
    P[0] = cm(cm(u0, U(Lu[n][1][ly][lz])), cc(cm(U(Lu[c][0][ly + 1][lz]), u1)));
    P[1] = cm(cm(u0, U(Lu[n][2][ly][lz])), cc(cm(U(Lu[c][0][ly][lz + 1]), u2)));
    P[2] = cm(cm(u1, U(Lu[c][2][ly + 1][lz])), cc(cm(U(Lu[c][1][ly][lz + 1]), u2)));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sn[k] = P[k].y;
      om[k] = P[k].x >= T(0) ? quot_t(P[k].y * P[k].y, T(1) + P[k].x) : T(1) - P[k].x;
    }
  };

  double acc[kU1Acc];
#pragma unroll
  for (int k = 0; k < kU1Acc; ++k) acc[k] = 0.0;

  // registers: plane x-1 (own column) and raw momenta of planes x, x+1
  T pm[2][RY], s01m[RY], s02m[RY];
  C2<T> um[RY];  // U_0 - 1 of the own column at plane x-1
  T qc[5][RY], qn[5][RY];

  // prologue: plane x0-1 -> buffer 1, plane x0 -> buffer 0; S_01, S_02 of
  // plane x0-1; then plane x0+1 -> buffer 1
  drift_into(1);
  load_plane(x0);
  drift_into(0);
#pragma unroll
  for (int r = 0; r < RY; ++r)
#pragma unroll
    for (int c = 0; c < 5; ++c) qc[c][r] = raw[c < 2 ? 2 + c : 5 + c][r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int ly = 1 + r * BY + ty, lz = 1 + tz;
    T sn[3], om[3];
    plaq(1, 0, ly, lz, sn, om);
    s01m[r] = sn[0];
    s02m[r] = sn[1];
    pm[0][r] = Lp[1][0][ly][lz];
    pm[1][r] = Lp[1][1][ly][lz];
    um[r] = Lu[1][0][ly][lz];
  }
  __syncthreads();
  load_plane((x0 + 1) % N);
  drift_into(1);
#pragma unroll
  for (int r = 0; r < RY; ++r)
#pragma unroll
    for (int c = 0; c < 5; ++c) qn[c][r] = raw[c < 2 ? 2 + c : 5 + c][r];

  for (int i = 0; i < A.XC; ++i) {
    const int x = x0 + i;
    const int cb_ = i & 1, nb_ = cb_ ^ 1;
    // plane x+2 is in flight during the compute below; the last iteration
    // re-reads plane x+1 (unused) so that the loads are unconditional and
    // the compiler need not wait for them at the first barrier
    load_plane(i + 1 < A.XC ? (x + 2) % N : (x + 1) % N);
    __syncthreads();
    // plaquette sines of the own sites and the low ring of plane x; the
    // handful of terms a thread adds per plane are summed in T, the running
    // sums over planes are FP64
    T mg = T(0);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ly = 1 + r * BY + ty, lz = 1 + tz;
      T sn[3], om[3];
      plaq(cb_, nb_, ly, lz, sn, om);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        Ls[k][ly][lz] = sn[k];
        mg += om[k];
      }
    }
    acc[7] += (double)mg;
    if (has_low) {
      T sn[3], om[3];
      plaq(cb_, nb_, sly, slz, sn, om);
#pragma unroll
      for (int k = 0; k < 3; ++k) Ls[k][sly][slz] = sn[k];
    }
    __syncthreads();
    // kick of the own sites of plane x
    T ts[kU1Acc];
#pragma unroll
    for (int k = 0; k < kU1Acc; ++k) ts[k] = T(0);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ly = 1 + r * BY + ty, lz = 1 + tz;
      const int o = site(x, y0 + r * BY + ty, z0 + tz);
      const C2<T> p{Lp[cb_][0][ly][lz], Lp[cb_][1][ly][lz]};
      const C2<T> fw[3] = {C2<T>{Lp[nb_][0][ly][lz], Lp[nb_][1][ly][lz]},
                           C2<T>{Lp[cb_][0][ly + 1][lz], Lp[cb_][1][ly + 1][lz]},
                           C2<T>{Lp[cb_][0][ly][lz + 1], Lp[cb_][1][ly][lz + 1]}};
      const C2<T> bw[3] = {C2<T>{pm[0][r], pm[1][r]}, C2<T>{Lp[cb_][0][ly - 1][lz], Lp[cb_][1][ly - 1][lz]},
                           C2<T>{Lp[cb_][0][ly][lz - 1], Lp[cb_][1][ly][lz - 1]}};
      const T th[3] = {Lt[cb_][0][ly][lz], Lt[cb_][1][ly][lz], Lt[cb_][2][ly][lz]};
      const C2<T> uf[3] = {Lu[cb_][0][ly][lz], Lu[cb_][1][ly][lz], Lu[cb_][2][ly][lz]};
      const C2<T> ub[3] = {um[r], Lu[cb_][1][ly - 1][lz], Lu[cb_][2][ly][lz - 1]};
      // covariant differences U phi_{+k} - phi = (U - 1) phi_{+k} + (phi_{+k} - phi):
      // both parts are small where the fields are smooth, so the FP32 result
      // keeps its relative precision instead of cancelling against the
      // condensate; the current Im[conj(phi) U phi_{+k}] = Im[conj(phi) g]
      C2<T> lap{T(0), T(0)};
      T Kcur[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const C2<T> uf1 = cm(uf[k], fw[k]);
        const C2<T> g{uf1.x + (fw[k].x - p.x), uf1.y + (fw[k].y - p.y)};
        const C2<T> ub1 = cm(cc(ub[k]), bw[k]);
        const C2<T> gb{ub1.x + (bw[k].x - p.x), ub1.y + (bw[k].y - p.y)};
        lap.x += g.x + gb.x;
        lap.y += g.y + gb.y;
        ts[2] += g.x * g.x + g.y * g.y;
        Kcur[k] = mul_c(cj, p.x * g.y - p.y * g.x);
      }
      const T r2 = p.x * p.x + p.y * p.y;
      // V'(phi) = (2 lambda |phi|^2 + m2) phi
      const C2<T> dvp{fma_c(lam2c, r2 * p.x, mul_c(m2c, p.x)), fma_c(lam2c, r2 * p.y, mul_c(m2c, p.y))};
      const C2<T> Kp{mul_c(cl, lap.x) - mul_c(cp, dvp.x), mul_c(cl, lap.y) - mul_c(cp, dvp.y)};
      const T S01 = Ls[0][ly][lz], S02 = Ls[1][ly][lz], S12 = Ls[2][ly][lz];
      const T curl[3] = {(S01 - Ls[0][ly - 1][lz]) + (S02 - Ls[1][ly][lz - 1]),
                         (-S01 + s01m[r]) + (S12 - Ls[2][ly][lz - 1]),
                         (-S02 + s02m[r]) + (-S12 + Ls[2][ly - 1][lz])};
      const C2<T> pin{qc[0][r], qc[1][r]};
      const C2<T> pout{fma_c(ck, Kp.x, pin.x), fma_c(ck, Kp.y, pin.y)};
      const C2<T> pe{fma_c(cE, Kp.x, pin.x), fma_c(cE, Kp.y, pin.y)};
      ts[0] += pin.x * pin.x + pin.y * pin.y;
      ts[1] += pe.x * pe.x + pe.y * pe.y;
      ts[3] += lam * r2 * r2;
      ts[4] += m2 * r2;
      ts[8] += p.x;
      ts[9] += p.y;
      ts[10] += r2;
      if (wr) {
        __builtin_nontemporal_store(p.x, &A.dst[0][o]);
        __builtin_nontemporal_store(p.y, &A.dst[1][o]);
        __builtin_nontemporal_store(pout.x, &A.dst[2][o]);
        __builtin_nontemporal_store(pout.y, &A.dst[3][o]);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T ain = qc[2 + k][r];
        const T KA = fma_c(cb, curl[k], Kcur[k]);
        const T aout = fma_c(ck, KA, ain), ae = fma_c(cE, KA, ain);
        ts[5] += ain * ain;
        ts[6] += ae * ae;
        if (wr) {
          __builtin_nontemporal_store(th[k], &A.dst[4 + k][o]);
          __builtin_nontemporal_store(aout, &A.dst[7 + k][o]);
        }
      }
      // plane x becomes plane x-1 of the next step
      pm[0][r] = p.x;
      pm[1][r] = p.y;
      um[r] = uf[0];
      s01m[r] = S01;
      s02m[r] = S02;
    }
#pragma unroll
    for (int k = 0; k < kU1Acc; ++k)
      if (k != 7) acc[k] += (double)ts[k];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        qc[c][r] = qn[c][r];
        qn[c][r] = raw[c < 2 ? 2 + c : 5 + c][r];
      }
    __syncthreads();
    if (i + 1 < A.XC) drift_into(cb_);  // plane x+2 replaces plane x
  }
  u1_block_partials<NT, kU1Acc>(acc, A.partials);
}

// Energies of Sec. 5.4.1 at a' from the lattice sums S of pass `pd`, which
// started from state `in`, and the scale-factor kernel with the gauge term
// (Sec. 5.1),
//   K_a = (1/3)(f/m_p)^2 a'^{1+2 alpha}[(alpha-2)E_K + alpha E_G + (alpha+1)E_V
//                                        + (alpha-1)(E_K^A + E_G^A)],
//   b_out = b + (wk1 + wk2) h K_a;  a, b, eta advanced when the pass updates.
// The state goes to `out` (may be `in`; nullptr: not stored); a and b after
// the pass are returned in a_next, b_next.
template <typename T>
__device__ void u1_finish_state(const U1PassArgs<T>& A, const PassDesc& pd, const DevState* in,
                                const double (&S)[kU1Acc], DevState* out, double& a_next, double& b_next) {
  constexpr int NACC = kU1Acc;
  const double V = (double)A.N * A.N * A.N;
  const double a_in = in->a, b_in = in->b, al = A.alpha;
  const double a = A.expand ? a_in + pd.wd * A.h * b_in : a_in;
  const bool lf = pd.mode == MODE_LF;
  const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2, dx2 = A.dx * A.dx;
  lattice_obs o;
  o.EK = (lf ? 0.5 * (S[0] + S[1]) : S[1]) / V / a6;
  o.EG = S[2] / V / (a2 * dx2);
  o.EV_term[0] = S[4] / V;
  o.EV_term[1] = S[3] / V;
  o.EV_term[2] = 0.0;
  o.EV = o.EV_term[0] + o.EV_term[1];
  o.EK_A = A.wf2 * (lf ? 0.5 * (S[5] + S[6]) : S[6]) / V / (2.0 * a4);
  o.EG_A = A.wf2 * S[7] / V / (a4 * dx2 * dx2 * A.e * A.e);
  o.EK_f[0] = o.EK;
  o.EK_f[1] = 0.0;
  o.EG_f[0] = o.EG;
  o.EG_f[1] = 0.0;
  o.mean_f[0] = S[8] / V;
  o.mean_f[1] = S[9] / V;
  o.meansq_f[0] = S[10] / V;
  o.meansq_f[1] = 0.0;
  bool bad = false;
  for (int k = 0; k < NACC; ++k) bad = bad || !isfinite(S[k]);
  const double rho = o.EK + o.EG + o.EV + o.EK_A + o.EG_A;
  double b_out = b_in, b_sync = b_in, hc = 0.0;
  if (A.expand) {
    const double Ka = A.fmp2 / 3.0 * apow(a, 1.0 + 2.0 * al) *
                      ((al - 2.0) * o.EK + al * o.EG + (al + 1.0) * o.EV + (al - 1.0) * (o.EK_A + o.EG_A));
    b_out = b_in + (pd.wk1 + pd.wk2) * A.h * Ka;
    b_sync = lf ? 0.5 * (b_in + b_out) : b_in + pd.wk1 * A.h * Ka;
    const double rhs = A.fmp2 / 3.0 * apow(a, 2.0 * (al + 1.0)) * rho;
    hc = fabs(b_sync * b_sync - rhs) / (b_sync * b_sync);
  }
  const double eta_new = in->eta + pd.wd * A.h;
  o.eta = eta_new;
  o.a = a;
  o.b = b_sync;
  o.H = b_sync / a;
  o.rho = rho;
  o.p = o.EK - o.EG / 3.0 - o.EV + (o.EK_A + o.EG_A) / 3.0;
  o.w = rho != 0.0 ? o.p / rho : 0.0;
  o.hc = hc;
  o.gauss = in->obs.gauss;
  o.step = 0;
  o.staggered = lf ? 1 : 0;
  o.reserved = 0;
  a_next = pd.update ? a : a_in;
  b_next = pd.update ? b_out : b_in;
  if (!out) return;
  if (out != in) *out = *in;
  out->obs = o;
  if (bad) out->nonfinite = 1;
  if (pd.update) {
    out->a = a;
    out->b = b_out;
    out->eta = eta_new;
  }
}


// Sums of NB partial records in block order by one block of NT threads
// (strided per thread, then waves in order); thread 0 returns them in S.
template <int NT>
__device__ bool u1_reduce_partials(const double* partials, int nb, double (&S)[kU1Acc]) {
  // Thread t < NL reads doubles t, t + NL, t + 2 NL, ... of the nb records
  // laid end to end; NL is a multiple of the record length, so the loads are
  // coalesced and every value a thread reads belongs to accumulator t mod
  // NACC (reading whole records per thread touched a cache line per lane and
  // load).  The threads of each accumulator are then summed in thread order
  // by one lane each of the first wave: a fixed order, the same in every block.
  constexpr int NACC = kU1Acc, NL = (NT / NACC) * NACC;
  static_assert(NT >= 64 && NACC <= 64, "the first wave finishes the sums");
  __shared__ double red[NL];
  const int tid = threadIdx.x;
  const int64_t nv = (int64_t)nb * NACC;
  if (tid < NL) {
    double s = 0.0;
#pragma unroll 8
    for (int64_t e = tid; e < nv; e += NL) s += partials[e];
    red[tid] = s;
  }
  __syncthreads();
  if (tid >= 64) return false;
  double v = 0.0;
  if (tid < NACC)
    for (int j = tid; j < NL; j += NACC) v += red[j];
#pragma unroll
  for (int k = 0; k < NACC; ++k) S[k] = __shfl(v, k, 64);
  return tid == 0;
}

// The finish of the pass described by A, into `out`: one block of
// kU1FinishThreads threads (four waves leave each thread the registers for
// its FP64 sums; 1024 threads, held to 128 VGPRs, spilled them).
constexpr int kU1FinishThreads = 256;

template <typename T>
__global__ __launch_bounds__(kU1FinishThreads) void u1_pass_finish(U1PassArgs<T> A, int nblocks, DevState* out) {
  double S[kU1Acc];
  if (!u1_reduce_partials<kU1FinishThreads>(A.partials, nblocks, S)) return;
  double an, bn;
  u1_finish_state<T>(A, A.pd, A.st, S, out, an, bn);
}

template <typename T>
static void fill_args(lattice* h, U1Args<T>& A) {
  for (int c = 0; c < 10; ++c) A.c[c] = static_cast<T*>(h->buf[h->cur][c]);
  A.N = h->p.N;
  A.dx = h->dx;
  A.alpha = h->p.alpha;
  A.fmp2 = h->p.fstar_over_mp * h->p.fstar_over_mp;
  A.lam = h->p.lambda;
  A.m2 = h->p.m2[0];
  A.e = h->p.e;
  A.wf2 = h->p.omega_over_f * h->p.omega_over_f;
  A.h = h->p.dt;
  A.expand = h->p.expansion;
  A.partials = h->partials;
  A.st = h->st;
}

template <typename T>
static int u1_gauss_t(lattice* h) {
  U1Args<T> A;
  fill_args(h, A);
  const int64_t V = (int64_t)h->p.N * h->p.N * h->p.N;
  const int nb = (int)(V / 256);
  hipLaunchKernelGGL(u1_gauss_kernel<T>, dim3(nb), dim3(256), 0, h->stream, A);
  CL_HIP(hipGetLastError());
  hipLaunchKernelGGL(u1_gauss_finish_kernel, dim3(1), dim3(1024), 0, h->stream, h->partials, nb, h->st);
  CL_HIP(hipGetLastError());
  return LAT_OK;
}

// One pass from the current buffer into the other (or no stores for an
// observation), then the FP64 finish.
template <typename T, int TZ, int BY, int RY, bool NC>
static int u1_pass_t(lattice* h, const PassDesc& pd, PassChain* chain) {
  U1PassArgs<T> A;
  for (int c = 0; c < 10; ++c) {
    A.src[c] = static_cast<const T*>(h->buf[h->cur][c]);
    A.dst[c] = static_cast<T*>(h->buf[1 - h->cur][c]);
  }
  const int N = h->p.N;
  constexpr int TY = BY * RY;
  const int tiles = (N / TZ) * (N / TY);
  const int xc = h->tile.xc;
  A.N = N;
  A.XC = xc;
  const int nb = tiles * (N / xc);
  A.swizzle = (nb % 8 == 0) ? 1 : 0;
  A.dx = h->dx;
  A.alpha = h->p.alpha;
  A.fmp2 = h->p.fstar_over_mp * h->p.fstar_over_mp;
  A.lam = h->p.lambda;
  A.m2 = h->p.m2[0];
  A.e = h->p.e;
  A.wf2 = h->p.omega_over_f * h->p.omega_over_f;
  A.h = h->p.dt;
  A.expand = h->p.expansion;
  A.pd = pd;
  A.partials = h->partials;
  A.st = h->st;
  A.prev = PrevPass{};
  DevState* slot[2] = {h->st, h->st2};
  if (chain) {
    A.st = slot[chain->rd];
    A.partials = (chain->k & 1) ? h->partials2 : h->partials;
    A.prev = chain->prev;
    if (A.prev.partials) A.prev.out = slot[1 - chain->rd];
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (pd.write && 2 * h->timer_used + 1 < h->timer.size()) {
    ev0 = h->timer[2 * h->timer_used];
    ev1 = h->timer[2 * h->timer_used + 1];
    ++h->timer_used;
  }
  if (ev0)
    hipExtLaunchKernelGGL((u1_pass_kernel<T, TZ, BY, RY, NC>), dim3(nb), dim3(TZ * BY), 0, h->stream, ev0, ev1, 0,
                          A);
  else
    hipLaunchKernelGGL((u1_pass_kernel<T, TZ, BY, RY, NC>), dim3(nb), dim3(TZ * BY), 0, h->stream, A);
  CL_HIP(hipGetLastError());
  if (chain) {
    if (A.prev.partials) chain->rd ^= 1;
    chain->prev = PrevPass{A.partials, nb, pd, nullptr};
    ++chain->k;
  } else {
    hipLaunchKernelGGL(u1_pass_finish<T>, dim3(1), dim3(kU1FinishThreads), 0, h->stream, A, nb, h->st);
    CL_HIP(hipGetLastError());
  }
  if (pd.write) h->cur ^= 1;
  return LAT_OK;
}

// Trailing finish of a chain: the last pass's records, from the slot that
// pass started from, into h->st.
template <typename T>
static int u1_chain_finish(lattice* h, const PassChain& c) {
  U1PassArgs<T> A = {};
  A.N = h->p.N;
  A.dx = h->dx;
  A.alpha = h->p.alpha;
  A.fmp2 = h->p.fstar_over_mp * h->p.fstar_over_mp;
  A.lam = h->p.lambda;
  A.m2 = h->p.m2[0];
  A.e = h->p.e;
  A.wf2 = h->p.omega_over_f * h->p.omega_over_f;
  A.h = h->p.dt;
  A.expand = h->p.expansion;
  A.pd = c.prev.pd;
  A.partials = const_cast<double*>(c.prev.partials);
  A.st = c.rd ? h->st2 : h->st;
  hipLaunchKernelGGL(u1_pass_finish<T>, dim3(1), dim3(kU1FinishThreads), 0, h->stream, A, c.prev.nblocks, h->st);
  CL_HIP(hipGetLastError());
  return LAT_OK;
}

// Compiled tile shapes of the U(1) pass (256 threads each): TZ x (BY RY) sites.
static const int kU1Shapes32[][3] = {{64, 4, 2}, {32, 8, 1}};
static const int kU1Shapes64[][3] = {{32, 8, 1}};

int u1_num_shapes(int fp32) { return fp32 ? 2 : 1; }
void u1_get_shape(int fp32, int i, int* tz, int* by, int* ry) {
  const int* s = fp32 ? kU1Shapes32[i] : kU1Shapes64[i];
  *tz = s[0];
  *by = s[1];
  *ry = s[2];
}

// Shape and x-chunk from h->tile (checked by tiling_ok).
template <bool NC>
static int u1_pass_nc(lattice* h, const PassDesc& pd, PassChain* chain) {
  const Tiling& t = h->tile;
  if (h->p.precision == LAT_FP32) {
    if (t.tz == 64 && t.by == 4 && t.ry == 2) return u1_pass_t<float, 64, 4, 2, NC>(h, pd, chain);
    if (t.tz == 32 && t.by == 8 && t.ry == 1) return u1_pass_t<float, 32, 8, 1, NC>(h, pd, chain);
  } else if (t.tz == 32 && t.by == 8 && t.ry == 1) {
    return u1_pass_t<double, 32, 8, 1, NC>(h, pd, chain);
  }
  set_error("U(1) pass: tile shape not compiled");
  return LAT_EINVAL;
}

int u1_pass(lattice* h, const PassDesc& pd, PassChain* chain) {
  if (h->p.model == LAT_MODEL_U1_NC) return u1_pass_nc<true>(h, pd, chain);
  return u1_pass_nc<false>(h, pd, chain);
}

int u1_gauss(lattice* h) { return h->p.precision == LAT_FP32 ? u1_gauss_t<float>(h) : u1_gauss_t<double>(h); }

// The pass sequence of the scalar path (merged kicks; leapfrog start-up,
// drift+kick passes and closing drift), run with the U(1) pass.
int u1_chain_end(lattice* h, const PassChain& chain) {
  if (chain.k == 0) return LAT_OK;
  return h->p.precision == LAT_FP32 ? u1_chain_finish<float>(h, chain) : u1_chain_finish<double>(h, chain);
}

int u1_step(lattice* h, int64_t n) {
  const std::vector<PassDesc> sched = pass_schedule(h->p.integrator, h->weights, &h->staggered, n);
  PassChain chain;
  for (const PassDesc& pd : sched) {
    const int rc = u1_pass(h, pd, &chain);
    if (rc) return rc;
  }
  const int rc = u1_chain_end(h, chain);
  if (rc) return rc;
  h->step += n;
  return LAT_OK;
}

// ---------------------------------------------------------------------------
// initial state (Sec. 7.2)
// ---------------------------------------------------------------------------
struct U1ModeArgs {
  int N, comp, deriv;
  uint64_t seed;
  double kIR, P0, a, alpha, m2eff, Hhom, kcut;
};

__device__ __forceinline__ int wrapk_u1(int i, int N) { return i <= N / 2 ? i : i - N; }

// Modes of the real component `comp` of phi = (phi_0 + i phi_1)/sqrt 2 with the
// zero-charge constraints |l_n| = |r_n|, th_1^r = th_0^r + th_1^l - th_0^l.
// Philox(counter = (lin, n, 0), key = seed): u0 -> |l_n| (Rayleigh, E|.|^2 = P),
// u2 -> th_n^l, u3 of component 0 -> th_0^r.
__global__ void u1_modes_kernel(double2* F, U1ModeArgs M) {
  const int64_t V = (int64_t)M.N * M.N * M.N;
  const int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lin >= V) return;
  const int N = M.N;
  const int i3 = (int)(lin % N), i2 = (int)((lin / N) % N), i1 = (int)(lin / ((int64_t)N * N));
  const int64_t par = ((int64_t)((N - i1) % N) * N + (N - i2) % N) * N + (N - i3) % N;
  if (lin > par) return;
  if (lin == par) { F[lin] = make_double2(0.0, 0.0); return; }
  const int n1 = wrapk_u1(i1, N), n2 = wrapk_u1(i2, N), n3 = wrapk_u1(i3, N);
  const double k = M.kIR * sqrt((double)n1 * n1 + (double)n2 * n2 + (double)n3 * n3);
  const double om2 = k * k + M.a * M.a * M.m2eff;
  if (!(om2 > 0.0) || (M.kcut > 0.0 && k > M.kcut)) {
    F[lin] = make_double2(0.0, 0.0);
    F[par] = make_double2(0.0, 0.0);
    return;
  }
  const double om = sqrt(om2), P = M.P0 / (2.0 * M.a * M.a * om);
  const uint32_t k0 = (uint32_t)M.seed, k1 = (uint32_t)(M.seed >> 32);
  const uint32_t c0 = (uint32_t)lin, c1 = (uint32_t)((uint64_t)lin >> 32);
  const Philox4 un = philox4x32_10(c0, c1, (uint32_t)M.comp, 0u, k0, k1);
  const Philox4 u0 = philox4x32_10(c0, c1, 0u, 0u, k0, k1);
  const double two32 = 4294967296.0, twopi = 6.283185307179586476925286766559;
  const double R = sqrt(-P * log(((double)un.v[0] + 0.5) / two32));
  const double thl = twopi * ((double)un.v[2] + 0.5) / two32;
  const double th0l = twopi * ((double)u0.v[2] + 0.5) / two32;
  const double th0r = twopi * ((double)u0.v[3] + 0.5) / two32;
  const double thr = M.comp == 0 ? th0r : th0r + thl - th0l;
  double sl, cl_, sr, cr;
  sincos(thl, &sl, &cl_);
  sincos(thr, &sr, &cr);
  const double Lx = R * cl_, Ly = R * sl, Rx = R * cr, Ry = R * sr;
  const double is2 = 0.70710678118654752440084436210485;
  double2 v;
  if (!M.deriv) {
    v = make_double2((Lx + Rx) * is2, (Ly + Ry) * is2);
  } else {
    const double c = apow(M.a, -(1.0 - M.alpha)) * om * is2;
    v = make_double2(-c * (Ly - Ry) - M.Hhom * (Lx + Rx) * is2, c * (Lx - Rx) - M.Hhom * (Ly + Ry) * is2);
  }
  F[lin] = v;
  F[par] = make_double2(v.x, -v.y);
}

__global__ void u1_take_real_kernel(const double2* F, double* out, int64_t V, double base, double invV) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < V) out[i] = base + F[i].x * invV;
}

// phi = (phi_0 + i phi_1)/sqrt 2, pi = a^{3-alpha}(phi_0' + i phi_1')/sqrt 2, and the
// charge density rho = 2e (f/w)^2 Im[conj phi pi] (FP64, from the unrounded values)
template <typename T>
__global__ void u1_store_kernel(const double* f0, const double* f1, const double* d0, const double* d1, T* pr,
                                T* pim, T* qr, T* qim, double2* rho, int64_t V, double cpi, double cq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const double is2 = 0.70710678118654752440084436210485;
  const double a = f0[i] * is2, b = f1[i] * is2, c = cpi * d0[i] * is2, d = cpi * d1[i] * is2;
  pr[i] = (T)a;
  pim[i] = (T)b;
  qr[i] = (T)c;
  qim[i] = (T)d;
  rho[i] = make_double2(cq * (a * d - b * c), 0.0);
}

// Minimum-norm solution of sum_i s_i E_i = rho^ with s_i = (1 - e^{+2 pi i n_i/N})/dx:
// E_i = conj(s_i) rho^ / sum_j |s_j|^2, E(0) = 0.
__global__ void u1_gauss_solve_kernel(const double2* R, double2* F, int N, int dir, double dx) {
  const int64_t V = (int64_t)N * N * N;
  const int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lin >= V) return;
  const int idx[3] = {(int)(lin / ((int64_t)N * N)), (int)((lin / N) % N), (int)(lin % N)};
  const double twopi = 6.283185307179586476925286766559;
  double den = 0.0, sr = 0.0, si = 0.0;
  for (int j = 0; j < 3; ++j) {
    double sn, cs;
    sincos(twopi * (double)idx[j] / (double)N, &sn, &cs);
    const double xr = (1.0 - cs) / dx, xi = -sn / dx;
    den += xr * xr + xi * xi;
    if (j == dir) { sr = xr; si = xi; }
  }
  if (den == 0.0) { F[lin] = make_double2(0.0, 0.0); return; }
  const double2 r = R[lin];
  // conj(s) * r = (sr - i si)(r.x + i r.y)
  F[lin] = make_double2((sr * r.x + si * r.y) / den, (sr * r.y - si * r.x) / den);
}

template <typename T>
__global__ void u1_store_link_momentum_kernel(const double2* F, T* out, int64_t V, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < V) out[i] = (T)(scale * F[i].x);
}

template <typename T>
__global__ void u1_zero_phases_kernel(T* t0, T* t1, T* t2, int64_t V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  t0[i] = t1[i] = t2[i] = T(0);
}

// Real component `comp` (0..3) of a charged scalar, or its derivative, into
// out (V doubles): base plus the inverse DFT of the vacuum modes of Sec. 7.2
// with the zero-charge constraints (or base alone for LAT_IC_HOMOGENEOUS).
int charged_mode_field(lattice* h, int comp, int deriv, double m2eff, double Hhom, double base, double* out) {
  const lattice_params& p = h->p;
  const int N = p.N;
  const int64_t V = (int64_t)N * N * N;
  double2* F = reinterpret_cast<double2*>(h->fft);
  const int thr = 256;
  const int blk = (int)((V + thr - 1) / thr);
  if (p.ic == LAT_IC_VACUUM) {
    U1ModeArgs M;
    M.N = N;
    M.comp = comp;
    M.deriv = deriv;
    M.seed = p.seed;
    M.kIR = p.kIR;
    M.P0 = p.omega_over_f * p.omega_over_f * std::pow((double)N / h->dx, 3.0);
    M.a = p.a0;
    M.alpha = p.alpha;
    M.m2eff = m2eff;
    M.Hhom = Hhom;
    M.kcut = p.kcut;
    hipLaunchKernelGGL(u1_modes_kernel, dim3(blk), dim3(thr), 0, h->stream, F, M);
    CL_HIP(hipGetLastError());
    int rc = run_fft3d(h, -1, 1.0);
    if (rc) return rc;
    hipLaunchKernelGGL(u1_take_real_kernel, dim3(blk), dim3(thr), 0, h->stream, F, out, V, base, 1.0 / (double)V);
  } else {
    hipLaunchKernelGGL(u1_take_real_kernel, dim3(blk), dim3(thr), 0, h->stream, F, out, V, base, 0.0);
  }
  CL_HIP(hipGetLastError());
  return LAT_OK;
}

// Minimum-norm solution of sum_i D-_i E_i = rho (Sec. 7.2) for the charge
// density whose DFT is R (V complex FP64, kept), into the three link-momentum
// components out[i] (storage precision: fp32 selects float).
int gauss_solve_fields(lattice* h, const double2* R, void* const out[3], bool fp32) {
  const int N = h->p.N;
  const int64_t V = (int64_t)N * N * N;
  double2* F = reinterpret_cast<double2*>(h->fft);
  const int thr = 256;
  const int blk = (int)((V + thr - 1) / thr);
  for (int i = 0; i < 3; ++i) {
    hipLaunchKernelGGL(u1_gauss_solve_kernel, dim3(blk), dim3(thr), 0, h->stream, R, F, N, i, h->dx);
    CL_HIP(hipGetLastError());
    int rc = run_fft3d(h, -1, 1.0);
    if (rc) return rc;
    if (fp32)
      hipLaunchKernelGGL(u1_store_link_momentum_kernel<float>, dim3(blk), dim3(thr), 0, h->stream, F,
                         (float*)out[i], V, 1.0 / (double)V);
    else
      hipLaunchKernelGGL(u1_store_link_momentum_kernel<double>, dim3(blk), dim3(thr), 0, h->stream, F,
                         (double*)out[i], V, 1.0 / (double)V);
    CL_HIP(hipGetLastError());
  }
  return LAT_OK;
}

template <typename T>
static int u1_init_state_t(lattice* h) {
  const lattice_params& p = h->p;
  const int N = p.N;
  const int64_t V = (int64_t)N * N * N;
  const double a = p.a0, al = p.alpha, fmp2 = p.fstar_over_mp * p.fstar_over_mp;
  const double r2 = 0.5 * (p.phi0[0] * p.phi0[0] + p.phi0[1] * p.phi0[1]);
  const double rho_hom = (p.dphi0[0] * p.dphi0[0] + p.dphi0[1] * p.dphi0[1]) / (2.0 * std::pow(a, 2.0 * al)) +
                         p.lambda * r2 * r2 + p.m2[0] * r2;
  const double Hhom = p.expansion ? std::sqrt(fmp2 / 3.0 * std::pow(a, 2.0 * (al + 1.0)) * rho_hom) / a : 0.0;
  const double s = p.phi0[0] * p.phi0[0] + p.phi0[1] * p.phi0[1];
  double2* F = reinterpret_cast<double2*>(h->fft);
  double* scratch = reinterpret_cast<double*>(h->buf[1 - h->cur][0]);  // 4 V doubles, then rho^
  double* full[4] = {scratch, scratch + V, scratch + 2 * V, scratch + 3 * V};
  const int thr = 256;
  const int blk = (int)((V + thr - 1) / thr);
  for (int n = 0; n < 2; ++n) {
    for (int deriv = 0; deriv < 2; ++deriv) {
      double* out = full[deriv ? 2 + n : n];
      const double base = deriv ? p.dphi0[n] : p.phi0[n];
      if (p.ic == LAT_IC_VACUUM) {
        U1ModeArgs M;
        M.N = N;
        M.comp = n;
        M.deriv = deriv;
        M.seed = p.seed;
        M.kIR = p.kIR;
        M.P0 = p.omega_over_f * p.omega_over_f * std::pow((double)N / h->dx, 3.0);
        M.a = a;
        M.alpha = al;
        M.m2eff = p.lambda * (s + 2.0 * p.phi0[n] * p.phi0[n]) + p.m2[0];
        M.Hhom = Hhom;
        M.kcut = p.kcut;
        hipLaunchKernelGGL(u1_modes_kernel, dim3(blk), dim3(thr), 0, h->stream, F, M);
        CL_HIP(hipGetLastError());
        int rc = run_fft3d(h, -1, 1.0);
        if (rc) return rc;
        hipLaunchKernelGGL(u1_take_real_kernel, dim3(blk), dim3(thr), 0, h->stream, F, out, V, base,
                           1.0 / (double)V);
      } else {
        hipLaunchKernelGGL(u1_take_real_kernel, dim3(blk), dim3(thr), 0, h->stream, F, out, V, base, 0.0);
      }
      CL_HIP(hipGetLastError());
    }
  }
  T* c[10];
  for (int k = 0; k < 10; ++k) c[k] = static_cast<T*>(h->buf[h->cur][k]);
  const double cq = 2.0 * p.e / (p.omega_over_f * p.omega_over_f);
  hipLaunchKernelGGL(u1_store_kernel<T>, dim3(blk), dim3(thr), 0, h->stream, full[0], full[1], full[2], full[3],
                     c[0], c[1], c[2], c[3], F, V, std::pow(a, 3.0 - al), cq);
  CL_HIP(hipGetLastError());
  int rc = run_fft3d(h, +1, 1.0);
  if (rc) return rc;
  double2* R = reinterpret_cast<double2*>(scratch);
  CL_HIP(hipMemcpyAsync(R, F, (size_t)V * sizeof(double2), hipMemcpyDeviceToDevice, h->stream));
  for (int i = 0; i < 3; ++i) {
    hipLaunchKernelGGL(u1_gauss_solve_kernel, dim3(blk), dim3(thr), 0, h->stream, R, F, N, i, h->dx);
    CL_HIP(hipGetLastError());
    rc = run_fft3d(h, -1, 1.0);
    if (rc) return rc;
    // the kick conserves sum_i D-_i piA_i - rho(phi, pi) with no power of a,
    // so the momenta themselves solve the Gauss law at any a0 and alpha
    hipLaunchKernelGGL(u1_store_link_momentum_kernel<T>, dim3(blk), dim3(thr), 0, h->stream, F, c[7 + i], V,
                       1.0 / (double)V);
    CL_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(u1_zero_phases_kernel<T>, dim3(blk), dim3(thr), 0, h->stream, c[4], c[5], c[6], V);
  CL_HIP(hipGetLastError());
  rc = upload_scalars(h, a, 0.0, 0.0);
  if (rc) return rc;
  h->staggered = 0;
  h->step = 0;
  if (p.expansion) {
    rc = u1_energies(h);
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

// Magnetic field B_i on the sites (Sec. 5.4 observables), (i, j, k) cyclic.
// Compact: B_i = Im V_jk / (e dx^2) = sin(Phi_jk) / (e dx^2) with
// Phi_jk(n) = th_j(n) + th_k(n+j) - th_j(n+k) - th_k(n) from the stored
// phases; non-compact: B_i = D+_j A_k - D+_k A_j.  FP64 arithmetic on the
// stored values, the result in storage precision.
template <typename T, bool NC>
__global__ __launch_bounds__(256) void u1_magnetic_kernel(const T* lj, const T* lk, T* out, int N, int j, int k,
                                                          double e, double dx) {
  const size_t NN = (size_t)N * N;
  const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= NN * N) return;
  const int c[3] = {(int)(s / NN), (int)((s / N) % N), (int)(s % N)};
  auto plus = [&](int d) {
    int q[3] = {c[0], c[1], c[2]};
    q[d] = (q[d] + 1) % N;
    return (size_t)q[0] * NN + (size_t)q[1] * N + q[2];
  };
  const double vj = (double)lj[s], vk = (double)lk[s];
  const double vk_j = (double)lk[plus(j)], vj_k = (double)lj[plus(k)];
  double B;
  if constexpr (NC) {
    B = ((vk_j - vk) - (vj_k - vj)) / dx;
  } else {
    B = sin((vj + vk_j) - (vj_k + vk)) / (e * dx * dx);
  }
  out[s] = (T)B;
}

int u1_magnetic_field(lattice* h, int i, void* out) {
  const int N = h->p.N;
  const int64_t V = (int64_t)N * N * N;
  const int j = (i + 1) % 3, k = (i + 2) % 3;
  const void* lj = h->buf[h->cur][4 + j];
  const void* lk = h->buf[h->cur][4 + k];
  const dim3 grid((unsigned)((V + 255) / 256)), blk(256);
  const bool nc = h->p.model == LAT_MODEL_U1_NC;
  if (h->p.precision == LAT_FP32) {
    if (nc)
      hipLaunchKernelGGL((u1_magnetic_kernel<float, true>), grid, blk, 0, h->stream, (const float*)lj,
                         (const float*)lk, (float*)out, N, j, k, h->p.e, h->dx);
    else
      hipLaunchKernelGGL((u1_magnetic_kernel<float, false>), grid, blk, 0, h->stream, (const float*)lj,
                         (const float*)lk, (float*)out, N, j, k, h->p.e, h->dx);
  } else {
    if (nc)
      hipLaunchKernelGGL((u1_magnetic_kernel<double, true>), grid, blk, 0, h->stream, (const double*)lj,
                         (const double*)lk, (double*)out, N, j, k, h->p.e, h->dx);
    else
      hipLaunchKernelGGL((u1_magnetic_kernel<double, false>), grid, blk, 0, h->stream, (const double*)lj,
                         (const double*)lk, (double*)out, N, j, k, h->p.e, h->dx);
  }
  CL_HIP(hipGetLastError());
  return LAT_OK;
}

int u1_init_state(lattice* h) {
  return h->p.precision == LAT_FP32 ? u1_init_state_t<float>(h) : u1_init_state_t<double>(h);
}

int u1_energies(lattice* h) {
  int rc = u1_gauss(h);
  if (rc) return rc;
  if (h->staggered) return u1_pass(h, pass(0.0, 0.0, 1.0, MODE_LF, 0, 0));
  return u1_pass(h, pass(0.0, 0.0, 0.0, MODE_VV, 0, 0));
}

}  // namespace cl
