// Doublet with SU(2) x U(1) gauge links on gfx950 (Sec. 6: staggered
// leapfrog, velocity Verlet and its Yoshida compositions; initial state
// Sec. 7.2).  Every pass of the shared schedule is three kernels: a
// pointwise drift of the fields and links into the other state buffer, a
// kick of every momentum from the drifted fields with per-block FP64 partial
// sums, and the FP64 finish that advances a and b.
//
// Components (storage precision, N^3 each):
//   0..3   Phi = (Phi_0, Phi_1) as Re Phi_0, Im Phi_0, Re Phi_1, Im Phi_1
//          (Phi_c = (phi_2c + i phi_2c+1)/sqrt 2)
//   4..7   pi_Phi, same layout
//   8..10  phase th_i of the U(1) link V_i = exp(i th_i)
//   11..13 pi_A,i
//   14+4i+k  SU(2) link U_i = c0 + i c.sigma as (c0, c1, c2, c3)
//   26+3i+a  pi_B,i along T_a = sigma_a/2
// Kernels (forces of the lattice energies, the electric fields generating
// left multiplication of the links, U' = -i g dx pi_B U / a^{1-alpha}):
//   K_Phi   = a^{1+alpha} sum_i (W_i Phi_{+i} - 2 Phi + W_i(n-i)^dag Phi_{-i})/dx^2
//             - a^{3+alpha}(2 lambda |Phi|^2 + m2) Phi,   W_i = V_i U_i
//   K_A,i   = a^{1+alpha}(2e/dx)(f/w)^2 Im[Phi^dag W_i Phi_{+i}]
//             + a^{alpha-1}/(e dx^3) sum_{j!=i}(Im V_ij(n) - Im V_ij(n-j))
//   K_B,i^a = a^{1+alpha}(g/dx)(f/w)^2 Im[Phi^dag sigma_a W_i Phi_{+i}]
//             + a^{alpha-1} 2/(g dx^3) sum_{j!=i}(c_a[U_ij(n)] - c_a[U_j(n-j)^dag U_ij(n-j) U_j(n-j)])
// with c_a the vector part of an SU(2) element.  SU(2) elements are carried
// as quaternions (w, x, y, z) = w + i(x sigma_1 + y sigma_2 + z sigma_3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"
#include "phase.hpp"

namespace cl {

constexpr int kSu2Comp = 35;
constexpr int kPH = 0, kPI = 4, kTH = 8, kPA = 11, kUL = 14, kPB = 26;
constexpr int kSu2Acc = 16;  // the workspace reserves 16 FP64 partials per 256-site block
constexpr int kSu2GaussAcc = 6;

template <typename T>
struct Q4 {
  T w, x, y, z;
};
template <typename T>
struct Cx2 {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Q4<T> qmul(const Q4<T>& a, const Q4<T>& b) {
  // (a0 + i a.s)(b0 + i b.s) = a0 b0 - a.b + i (a0 b + b0 a - a x b).s
  return Q4<T>{a.w * b.w - (a.x * b.x + a.y * b.y + a.z * b.z),
               a.w * b.x + b.w * a.x - (a.y * b.z - a.z * b.y),
               a.w * b.y + b.w * a.y - (a.z * b.x - a.x * b.z),
               a.w * b.z + b.w * a.z - (a.x * b.y - a.y * b.x)};
}
template <typename T>
__device__ __forceinline__ Q4<T> qdag(const Q4<T>& a) {
  return Q4<T>{a.w, -a.x, -a.y, -a.z};
}
template <typename T>
__device__ __forceinline__ Cx2<T> cmul2(Cx2<T> a, Cx2<T> b) {
  return Cx2<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ Cx2<T> cadd2(Cx2<T> a, Cx2<T> b) {
  return Cx2<T>{a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ Cx2<T> csub2(Cx2<T> a, Cx2<T> b) {
  return Cx2<T>{a.re - b.re, a.im - b.im};
}
// the 2x2 matrix of (w, x, y, z) minus w1 times the identity, applied to a
// doublet: [[w - w1 + i z, y + i x], [-y + i x, w - w1 - i z]] (w1 = 0: the
// element itself, w1 = 1: the element minus one)
template <typename T>
__device__ __forceinline__ void qapply(const Q4<T>& q, T wm, const Cx2<T> (&v)[2], Cx2<T> (&o)[2]) {
  o[0] = cadd2(cmul2(Cx2<T>{wm, q.z}, v[0]), cmul2(Cx2<T>{q.y, q.x}, v[1]));
  o[1] = cadd2(cmul2(Cx2<T>{-q.y, q.x}, v[0]), cmul2(Cx2<T>{wm, -q.z}, v[1]));
}
// w - 1 of a unit quaternion without cancellation: -|v|^2/(1 + w) for w > 0
template <typename T>
__device__ __forceinline__ T qw_m1(const Q4<T>& q) {
  const T v2 = q.x * q.x + q.y * q.y + q.z * q.z;
  return q.w > T(0) ? -v2 / (T(1) + q.w) : q.w - T(1);
}
// Im(conj(a) b), Re(conj(a) b)
template <typename T>
__device__ __forceinline__ T cross_im(Cx2<T> a, Cx2<T> b) { return a.re * b.im - a.im * b.re; }
template <typename T>
__device__ __forceinline__ T dot_re(Cx2<T> a, Cx2<T> b) { return a.re * b.re + a.im * b.im; }

__device__ __forceinline__ float rsqrt_s(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_s(double x) { return 1.0 / sqrt(x); }

template <typename T>
__device__ __forceinline__ T wrap_turns(T t) {
  const T twopi = (T)6.283185307179586476925286766559;
  return t - twopi * rint(t * (T)0.15915494309189533576888376337251);
}

template <typename T>
struct Su2Args {
  const T* src[kSu2Comp];
  T* dst[kSu2Comp];
  int N;
  double dx, alpha, fmp2, lam, m2, e, g, wf2, h;
  int expand;
  int fields_in_dst;  // the kick reads the drifted fields from dst (else src)
  PassDesc pd;
  double* partials;
  DevState* st;
};

__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// per-block sums of 256 threads' accumulators (waves in order) into the block's record
template <int NACC>
__device__ void su2_block_partials(double (&acc)[NACC], double* partials) {
  __shared__ double red[4][NACC];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    const double s = wsum64(acc[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (tid < NACC) partials[(size_t)blockIdx.x * NACC + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// Drift of the fields and links into dst (Sec. 6.2.1 and 6.2.2):
//   Phi += wd h pi / a_mid^{3-alpha};
//   V   <- (1 - i u)/(1 + i u) V,  u = e wd h dx pi_A / (2 a_mid^{1-alpha}), as th -= 2 atan u;
//   U   <- (1 - i X)(1 + i X)^{-1} U = ((1 - |w|^2) - 2 i w.sigma)/(1 + |w|^2) U,
//          w = g wd h dx pi_B / (4 a_mid^{1-alpha});
// U is renormalised to unit length after the product (rounding only).
template <typename T>
__global__ __launch_bounds__(256) void su2_drift_kernel(Su2Args<T> A) {
  const size_t V = (size_t)A.N * A.N * A.N;
  const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= V) return;
  const double a_in = A.st->a, b_in = A.st->b;
  const double hw = A.pd.wd * A.h;
  const double anew = A.expand ? a_in + hw * b_in : a_in;
  const double amid = 0.5 * (a_in + anew);
  // coefficients as hi + lo pairs (no coherent rounding of them)
  const Coef<T> cd = ucoef<T>(hw * apow(amid, -(3.0 - A.alpha)));
  const Coef<T> cu = ucoef<T>(A.e * hw * A.dx / (2.0 * apow(amid, 1.0 - A.alpha)));
  const Coef<T> cw = ucoef<T>(A.g * hw * A.dx / (4.0 * apow(amid, 1.0 - A.alpha)));
#pragma unroll
  for (int k = 0; k < 4; ++k) A.dst[kPH + k][s] = fma_c(cd, A.src[kPI + k][s], A.src[kPH + k][s]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
    A.dst[kTH + i][s] = wrap_turns(A.src[kTH + i][s] - T(2) * atan_t(mul_c(cu, A.src[kPA + i][s])));
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const Q4<T> u{A.src[kUL + 4 * i][s], A.src[kUL + 4 * i + 1][s], A.src[kUL + 4 * i + 2][s],
                  A.src[kUL + 4 * i + 3][s]};
    const T w0 = mul_c(cw, A.src[kPB + 3 * i][s]), w1 = mul_c(cw, A.src[kPB + 3 * i + 1][s]),
            w2 = mul_c(cw, A.src[kPB + 3 * i + 2][s]);
    const T ww = w0 * w0 + w1 * w1 + w2 * w2;
    const T d = T(1) / (T(1) + ww);
    const Q4<T> c{(T(1) - ww) * d, T(-2) * w0 * d, T(-2) * w1 * d, T(-2) * w2 * d};
    Q4<T> n = qmul(c, u);
    const T r = rsqrt_s(n.w * n.w + n.x * n.x + n.y * n.y + n.z * n.z);
    A.dst[kUL + 4 * i][s] = n.w * r;
    A.dst[kUL + 4 * i + 1][s] = n.x * r;
    A.dst[kUL + 4 * i + 2][s] = n.y * r;
    A.dst[kUL + 4 * i + 3][s] = n.z * r;
  }
}

// Kick of every momentum at a' = a + wd h b from the (drifted) fields, and
// the lattice sums of the energies:
//   pi += (wk1 + wk2) h K; E_K from pi_in and pi + wk1 h K (VV) or the mean of
//   <pi_in^2> and <pi_out^2> (LF), for each of pi_Phi, pi_A, pi_B.
// Sums: 0,1 pi_Phi (in, e), 2 sum_i |W_i Phi_{+i} - Phi|^2, 3 lambda|Phi|^4,
// 4 m2|Phi|^2, 5,6 pi_A, 7 sum_{i<j}(1 - cos Phi_ij), 8,9 pi_B,
// 10 sum_{i<j}(1 - Re/Tr-half U_ij), 11..14 the four components of Phi, 15 |Phi|^2.
template <typename T>
__global__ __launch_bounds__(256, 2) void su2_kick_kernel(Su2Args<T> A) {
  const int N = A.N;
  const size_t NN = (size_t)N * N, V = NN * N;
  const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
  double acc[kSu2Acc];
#pragma unroll
  for (int k = 0; k < kSu2Acc; ++k) acc[k] = 0.0;
  if (s < V) {
    const T* const* F = A.fields_in_dst ? const_cast<const T* const*>(A.dst) : A.src;
    // periodic neighbour offsets, once per thread: sp[d] = n + e_d, sm[d] = n - e_d,
    // and dg[a][b] = n - e_b + e_a (a != b)
    // (sites fit in 32 bits: N^3 <= 2^30)
    const unsigned su = (unsigned)s, n = (unsigned)N, nn = (unsigned)NN;
    const unsigned c[3] = {su / nn, (su / n) % n, su % n};
    const unsigned str[3] = {nn, n, 1u};
    int op[3], om[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      op[d] = c[d] == n - 1 ? -(int)((n - 1) * str[d]) : (int)str[d];
      om[d] = c[d] == 0 ? (int)((n - 1) * str[d]) : -(int)str[d];
    }
    unsigned sp[3], sm[3], dg[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sp[d] = su + op[d];
      sm[d] = su + om[d];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) dg[a][b] = su + om[b] + op[a];
    auto LP = [&](unsigned t, Cx2<T> (&p)[2]) {
      p[0] = Cx2<T>{F[kPH][t], F[kPH + 1][t]};
      p[1] = Cx2<T>{F[kPH + 2][t], F[kPH + 3][t]};
    };
    auto LQ = [&](int i, unsigned t) -> Q4<T> {
      return Q4<T>{F[kUL + 4 * i][t], F[kUL + 4 * i + 1][t], F[kUL + 4 * i + 2][t], F[kUL + 4 * i + 3][t]};
    };
    auto LT = [&](int i, unsigned t) -> T { return F[kTH + i][t]; };

    const double a_in = A.st->a, b_in = A.st->b;
    const double anew = A.expand ? a_in + A.pd.wd * A.h * b_in : a_in;
    const Coef<T> cl = ucoef<T>(apow(anew, 1.0 + A.alpha) / (A.dx * A.dx));
    const Coef<T> cp = ucoef<T>(apow(anew, 3.0 + A.alpha));
    const Coef<T> cjA = ucoef<T>(apow(anew, 1.0 + A.alpha) * 2.0 * A.e / A.dx / A.wf2);
    const Coef<T> cjB = ucoef<T>(apow(anew, 1.0 + A.alpha) * A.g / A.dx / A.wf2);
    const Coef<T> cbA = ucoef<T>(apow(anew, A.alpha - 1.0) / (A.e * A.dx * A.dx * A.dx));
    const Coef<T> cbB = ucoef<T>(apow(anew, A.alpha - 1.0) * 2.0 / (A.g * A.dx * A.dx * A.dx));
    const Coef<T> ck = ucoef<T>((A.pd.wk1 + A.pd.wk2) * A.h);
    const Coef<T> cE = ucoef<T>((A.pd.mode == MODE_LF ? A.pd.wk1 + A.pd.wk2 : A.pd.wk1) * A.h);
    const T lam = (T)A.lam, m2 = (T)A.m2;
    const Coef<T> lam2c = ucoef<T>(2.0 * A.lam), m2c = ucoef<T>(A.m2);

    Cx2<T> p[2];
    LP(su, p);
    // ---- matter: covariant differences in the cancellation-free form
    //   W Phi_+ - Phi = (V - 1) y + (U - 1) Phi_+ + (Phi_+ - Phi),  y = U Phi_+
    //   W(n-i)^dag Phi_- - Phi = (U^dag - 1) y' + (conj V - 1) Phi_- + (Phi_- - Phi),  y' = conj(V) Phi_-
    Cx2<T> lap[2] = {{T(0), T(0)}, {T(0), T(0)}};
    T eg = T(0), curA[3], curB[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Cx2<T> fp[2], fm[2];
      LP(sp[i], fp);
      LP(sm[i], fm);
      // forward
      const Q4<T> u = LQ(i, su);
      Cx2<T> um1f[2];
      qapply(u, qw_m1(u), fp, um1f);  // (U - 1) Phi_+
      T sn, cm;
      sincos_m1(LT(i, su), &sn, &cm);
      const Cx2<T> vm1{cm, sn};
      Cx2<T> g[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const Cx2<T> y = cadd2(fp[k], um1f[k]);
        g[k] = cadd2(cadd2(cmul2(vm1, y), um1f[k]), csub2(fp[k], p[k]));
      }
      // backward
      const Q4<T> ub = qdag(LQ(i, sm[i]));
      T snb, cmb;
      sincos_m1(LT(i, sm[i]), &snb, &cmb);
      const Cx2<T> vbm1{cmb, -snb};  // conj(V) - 1
      Cx2<T> vf[2], yb[2], ubm1[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        vf[k] = cmul2(vbm1, fm[k]);
        yb[k] = cadd2(fm[k], vf[k]);
      }
      qapply(ub, qw_m1(ub), yb, ubm1);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const Cx2<T> gb = cadd2(cadd2(ubm1[k], vf[k]), csub2(fm[k], p[k]));
        lap[k] = cadd2(lap[k], cadd2(g[k], gb));
      }
      eg += g[0].re * g[0].re + g[0].im * g[0].im + g[1].re * g[1].re + g[1].im * g[1].im;
      // currents Im[Phi^dag g], Im[Phi^dag sigma_a g] (Im[Phi^dag sigma Phi] = 0)
      curA[i] = cross_im(p[0], g[0]) + cross_im(p[1], g[1]);
      curB[i][0] = cross_im(p[0], g[1]) + cross_im(p[1], g[0]);
      curB[i][1] = -dot_re(p[0], g[1]) + dot_re(p[1], g[0]);
      curB[i][2] = cross_im(p[0], g[0]) - cross_im(p[1], g[1]);
    }
    const T r2 = p[0].re * p[0].re + p[0].im * p[0].im + p[1].re * p[1].re + p[1].im * p[1].im;

    // ---- U(1) plaquettes: sin Phi_ab(m), Phi_ab(m) = th_a(m) + th_b(m+a) - th_a(m+b) - th_b(m),
    // at m = n and at m = n - e_q (m + e_a = n when a = q)
    auto pos = [&](int q, int a) -> unsigned { return a == q ? su : dg[a][q]; };
    auto plA = [&](int a, int b, int q, T* om1) -> T {
      const unsigned m = q < 0 ? su : sm[q];
      const unsigned ma = q < 0 ? sp[a] : pos(q, a), mb = q < 0 ? sp[b] : pos(q, b);
      const T ph = (LT(a, m) + LT(b, ma)) - (LT(a, mb) + LT(b, m));
      T sn, cm;
      sincos_m1(ph, &sn, &cm);
      if (om1) *om1 = -cm;  // 1 - cos Phi
      return sn;
    };
    T omA[3];
    const T S01 = plA(0, 1, -1, &omA[0]), S02 = plA(0, 2, -1, &omA[1]), S12 = plA(1, 2, -1, &omA[2]);
    const T curlA[3] = {(S01 - plA(0, 1, 1, nullptr)) + (S02 - plA(0, 2, 2, nullptr)),
                        (-S01 + plA(0, 1, 0, nullptr)) + (S12 - plA(1, 2, 2, nullptr)),
                        (-S02 + plA(0, 2, 0, nullptr)) + (-S12 + plA(1, 2, 1, nullptr))};

    // ---- SU(2) plaquettes U_ab(n) = U_a(n) U_b(n+a) U_a(n+b)^dag U_b(n)^dag and the
    // backward ones transported to n (products of three links)
    auto plB = [&](int a, int b) -> Q4<T> {
      return qmul(qmul(LQ(a, su), LQ(b, sp[a])), qdag(qmul(LQ(b, su), LQ(a, sp[b]))));
    };
    const Q4<T> P01 = plB(0, 1), P02 = plB(0, 2), P12 = plB(1, 2);
    T omB = T(0);
    {
      const Q4<T>* P[3] = {&P01, &P02, &P12};
#pragma unroll
      for (int k = 0; k < 3; ++k) omB += -qw_m1(*P[k]);  // 1 - w = (2 - Tr)/2
    }
    // i = a, plane (a, b), base m = n - b: U_b(m)^dag U_a(m) U_b(m+a) U_a(n)^dag
    auto tA = [&](int a, int b) -> Q4<T> {
      return qmul(qmul(qdag(LQ(b, sm[b])), LQ(a, sm[b])), qmul(LQ(b, dg[a][b]), qdag(LQ(a, su))));
    };
    // i = b, plane (a, b), base m = n - a: U_b(n) U_a(m+b)^dag U_b(m)^dag U_a(m)
    auto tB = [&](int a, int b) -> Q4<T> {
      return qmul(qmul(LQ(b, su), qdag(LQ(a, dg[b][a]))), qmul(qdag(LQ(b, sm[a])), LQ(a, sm[a])));
    };
    T magB[3][3];
    {
      const Q4<T> t01 = tA(0, 1), t02 = tA(0, 2), t12 = tA(1, 2);
      const Q4<T> r01 = tB(0, 1), r02 = tB(0, 2), r12 = tB(1, 2);
      // i = 0: [c(P01) - c(t01)] + [c(P02) - c(t02)]
      magB[0][0] = (P01.x - t01.x) + (P02.x - t02.x);
      magB[0][1] = (P01.y - t01.y) + (P02.y - t02.y);
      magB[0][2] = (P01.z - t01.z) + (P02.z - t02.z);
      // i = 1: [-c(P01) + c(r01)] + [c(P12) - c(t12)]
      magB[1][0] = (r01.x - P01.x) + (P12.x - t12.x);
      magB[1][1] = (r01.y - P01.y) + (P12.y - t12.y);
      magB[1][2] = (r01.z - P01.z) + (P12.z - t12.z);
      // i = 2: [-c(P02) + c(r02)] + [-c(P12) + c(r12)]
      magB[2][0] = (r02.x - P02.x) + (r12.x - P12.x);
      magB[2][1] = (r02.y - P02.y) + (r12.y - P12.y);
      magB[2][2] = (r02.z - P02.z) + (r12.z - P12.z);
    }

    // ---- kicks and sums
    const bool wr = A.pd.write != 0;
    T ts[kSu2Acc];
#pragma unroll
    for (int k = 0; k < kSu2Acc; ++k) ts[k] = T(0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      // V'(Phi) = (2 lambda |Phi|^2 + m2) Phi
      const T dre = fma_c(lam2c, r2 * p[k].re, mul_c(m2c, p[k].re));
      const T dim = fma_c(lam2c, r2 * p[k].im, mul_c(m2c, p[k].im));
      const Cx2<T> K{mul_c(cl, lap[k].re) - mul_c(cp, dre), mul_c(cl, lap[k].im) - mul_c(cp, dim)};
      const Cx2<T> pin{A.src[kPI + 2 * k][s], A.src[kPI + 2 * k + 1][s]};
      const Cx2<T> pe{fma_c(cE, K.re, pin.re), fma_c(cE, K.im, pin.im)};
      ts[0] += pin.re * pin.re + pin.im * pin.im;
      ts[1] += pe.re * pe.re + pe.im * pe.im;
      if (wr) {
        A.dst[kPI + 2 * k][s] = fma_c(ck, K.re, pin.re);
        A.dst[kPI + 2 * k + 1][s] = fma_c(ck, K.im, pin.im);
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T K = fma_c(cbA, curlA[i], mul_c(cjA, curA[i]));
      const T ain = A.src[kPA + i][s], ae = fma_c(cE, K, ain);
      ts[5] += ain * ain;
      ts[6] += ae * ae;
      if (wr) A.dst[kPA + i][s] = fma_c(ck, K, ain);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T KB = fma_c(cbB, magB[i][a], mul_c(cjB, curB[i][a]));
        const T bin = A.src[kPB + 3 * i + a][s], be = fma_c(cE, KB, bin);
        ts[8] += bin * bin;
        ts[9] += be * be;
        if (wr) A.dst[kPB + 3 * i + a][s] = fma_c(ck, KB, bin);
      }
    }
    if (wr && !A.fields_in_dst) {
      // a kick-only pass: the fields move to the other buffer unchanged
#pragma unroll
      for (int k = 0; k < 4; ++k) A.dst[kPH + k][s] = A.src[kPH + k][s];
#pragma unroll
      for (int i = 0; i < 3; ++i) A.dst[kTH + i][s] = A.src[kTH + i][s];
#pragma unroll
      for (int k = 0; k < 12; ++k) A.dst[kUL + k][s] = A.src[kUL + k][s];
    }
    ts[2] = eg;
    ts[3] = lam * r2 * r2;
    ts[4] = m2 * r2;
    ts[7] = omA[0] + omA[1] + omA[2];
    ts[10] = omB;
    ts[11] = p[0].re;
    ts[12] = p[0].im;
    ts[13] = p[1].re;
    ts[14] = p[1].im;
    ts[15] = r2;
#pragma unroll
    for (int k = 0; k < kSu2Acc; ++k) acc[k] = (double)ts[k];
  }
  su2_block_partials<kSu2Acc>(acc, A.partials);
}

// Energies (Sec. 5.4.1, Sec. 6.3.1) at a' and the scale-factor kernel with
// both gauge sectors, K_a = (1/3)(f/m_p)^2 a'^{1+2 alpha}[(alpha-2)E_K + alpha E_G
// + (alpha+1)E_V + (alpha-1)(E_K^A + E_G^A + E_K^B + E_G^B)]; b_out = b + (wk1 + wk2) h K_a.
// First stage of a pass's reduction: block g of R sums the contiguous range
// g of the nb records (lanes in order, then the waves in order) into record g
// of `out`, so that the one-block finish reads R records, not nb.  With one
// block reading the 8192 records of a 128^3 pass the finish took 36 us.
constexpr int kSu2FoldBlocks = 64;

template <int NACC>
__global__ __launch_bounds__(256) void su2_fold_records(const double* in, int nb, double* out) {
  __shared__ double red[4][NACC];
  const int R = gridDim.x, g = blockIdx.x;
  const int chunk = (nb + R - 1) / R;
  const int b0 = g * chunk, b1 = b0 + chunk < nb ? b0 + chunk : nb;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double t[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) t[k] = 0.0;
  for (int b = b0 + tid; b < b1; b += 256)
#pragma unroll
    for (int k = 0; k < NACC; ++k) t[k] += in[(size_t)b * NACC + k];
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    const double v = wsum64(t[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (tid < NACC) out[(size_t)g * NACC + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// One block of kSu2FinishThreads threads: four waves leave each thread the
// registers for its FP64 sums (1024 threads, held to 128 VGPRs, spilled them).
constexpr int kSu2FinishThreads = 256;

template <typename T>
__global__ __launch_bounds__(kSu2FinishThreads) void su2_finish_kernel(Su2Args<T> A, int nblocks) {
  constexpr int NW = kSu2FinishThreads / 64;
  __shared__ double red[NW][kSu2Acc];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double tot[kSu2Acc];
#pragma unroll
  for (int k = 0; k < kSu2Acc; ++k) tot[k] = 0.0;
  for (int b = tid; b < nblocks; b += kSu2FinishThreads)
#pragma unroll
    for (int k = 0; k < kSu2Acc; ++k) tot[k] += A.partials[(size_t)b * kSu2Acc + k];
#pragma unroll
  for (int k = 0; k < kSu2Acc; ++k) {
    const double v = wsum64(tot[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  double S[kSu2Acc];
  for (int k = 0; k < kSu2Acc; ++k) {
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += red[w][k];
    S[k] = v;
  }
  const PassDesc& pd = A.pd;
  DevState* st = A.st;
  const double V = (double)A.N * A.N * A.N;
  const double a_in = st->a, b_in = st->b, al = A.alpha;
  const double a = A.expand ? a_in + pd.wd * A.h * b_in : a_in;
  const bool lf = pd.mode == MODE_LF;
  const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2, dx2 = A.dx * A.dx, dx4 = dx2 * dx2;
  lattice_obs o = st->obs;
  o.EK = (lf ? 0.5 * (S[0] + S[1]) : S[1]) / V / a6;
  o.EG = S[2] / V / (a2 * dx2);
  o.EV_term[0] = S[4] / V;
  o.EV_term[1] = S[3] / V;
  o.EV_term[2] = 0.0;
  o.EV = o.EV_term[0] + o.EV_term[1];
  o.EK_A = A.wf2 * (lf ? 0.5 * (S[5] + S[6]) : S[6]) / V / (2.0 * a4);
  o.EG_A = A.wf2 * S[7] / V / (a4 * dx4 * A.e * A.e);
  o.EK_B = A.wf2 * (lf ? 0.5 * (S[8] + S[9]) : S[9]) / V / (2.0 * a4);
  o.EG_B = 2.0 * A.wf2 * (2.0 * S[10]) / V / (a4 * dx4 * A.g * A.g);
  o.EK_f[0] = o.EK;
  o.EK_f[1] = 0.0;
  o.EG_f[0] = o.EG;
  o.EG_f[1] = 0.0;
  o.mean_f[0] = S[11] / V;
  o.mean_f[1] = S[12] / V;
  o.mean_lo[0] = S[13] / V;
  o.mean_lo[1] = S[14] / V;
  o.meansq_f[0] = S[15] / V;
  o.meansq_f[1] = 0.0;
  bool bad = false;
  for (int k = 0; k < kSu2Acc; ++k) bad = bad || !isfinite(S[k]);
  const double gauge = o.EK_A + o.EG_A + o.EK_B + o.EG_B;
  const double rho = o.EK + o.EG + o.EV + gauge;
  double b_out = b_in, b_sync = b_in, hc = 0.0;
  if (A.expand) {
    const double Ka = A.fmp2 / 3.0 * apow(a, 1.0 + 2.0 * al) *
                      ((al - 2.0) * o.EK + al * o.EG + (al + 1.0) * o.EV + (al - 1.0) * gauge);
    b_out = b_in + (pd.wk1 + pd.wk2) * A.h * Ka;
    b_sync = lf ? 0.5 * (b_in + b_out) : b_in + pd.wk1 * A.h * Ka;
    const double rhs = A.fmp2 / 3.0 * apow(a, 2.0 * (al + 1.0)) * rho;
    hc = fabs(b_sync * b_sync - rhs) / (b_sync * b_sync);
  }
  const double eta_new = st->eta + pd.wd * A.h;
  o.eta = eta_new;
  o.a = a;
  o.b = b_sync;
  o.H = b_sync / a;
  o.rho = rho;
  o.p = o.EK - o.EG / 3.0 - o.EV + gauge / 3.0;
  o.w = rho != 0.0 ? o.p / rho : 0.0;
  o.hc = hc;
  o.step = 0;
  o.staggered = lf ? 1 : 0;
  o.reserved = 0;
  st->obs = o;
  if (bad) st->nonfinite = 1;
  if (pd.update) {
    st->a = a;
    st->b = b_out;
    st->eta = eta_new;
  }
}

// Gauss residuals (Sec. 5.2 and Sec. 6.2, with the electric field at n - i
// transported to n):
//   G_A(n)   = sum_i (pi_A,i(n) - pi_A,i(n-i))/dx - 2e (f/w)^2 Im[Phi^dag pi]
//   G_B^a(n) = sum_i (pi_B,i(n) - U_i(n-i)^dag pi_B,i(n-i) U_i(n-i))^a/dx - g (f/w)^2 Im[Phi^dag sigma_a pi]
// in FP64 from the stored values.
template <typename T>
__global__ __launch_bounds__(256) void su2_gauss_kernel(Su2Args<T> A) {
  const int N = A.N;
  const size_t NN = (size_t)N * N, V = NN * N;
  const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
  double acc[kSu2GaussAcc] = {0, 0, 0, 0, 0, 0};
  if (s < V) {
    const T* const* F = A.src;
    const int c[3] = {(int)(s / NN), (int)((s / N) % N), (int)(s % N)};
    const size_t str[3] = {NN, (size_t)N, 1};
    double divA = 0.0, divB[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) {
      const size_t sm = c[i] > 0 ? s - str[i] : s + (size_t)(N - 1) * str[i];
      divA += ((double)F[kPA + i][s] - (double)F[kPA + i][sm]) / A.dx;
      const Q4<double> u{(double)F[kUL + 4 * i][sm], (double)F[kUL + 4 * i + 1][sm], (double)F[kUL + 4 * i + 2][sm],
                         (double)F[kUL + 4 * i + 3][sm]};
      // U^dag (x.sigma) U as the vector part of U^dag (0, x) U
      const Q4<double> xq{0.0, (double)F[kPB + 3 * i][sm], (double)F[kPB + 3 * i + 1][sm],
                          (double)F[kPB + 3 * i + 2][sm]};
      const Q4<double> t = qmul(qmul(qdag(u), xq), u);
      divB[0] += ((double)F[kPB + 3 * i][s] - t.x) / A.dx;
      divB[1] += ((double)F[kPB + 3 * i + 1][s] - t.y) / A.dx;
      divB[2] += ((double)F[kPB + 3 * i + 2][s] - t.z) / A.dx;
    }
    const Cx2<double> p0{(double)F[kPH][s], (double)F[kPH + 1][s]}, p1{(double)F[kPH + 2][s], (double)F[kPH + 3][s]};
    const Cx2<double> q0{(double)F[kPI][s], (double)F[kPI + 1][s]}, q1{(double)F[kPI + 2][s], (double)F[kPI + 3][s]};
    const double rhoA = 2.0 * A.e / A.wf2 * (cross_im(p0, q0) + cross_im(p1, q1));
    const double cB = A.g / A.wf2;
    const double rhoB[3] = {cB * (cross_im(p0, q1) + cross_im(p1, q0)), cB * (-dot_re(p0, q1) + dot_re(p1, q0)),
                            cB * (cross_im(p0, q0) - cross_im(p1, q1))};
    acc[0] = (divA - rhoA) * (divA - rhoA);
    acc[1] = divA * divA;
    acc[2] = rhoA * rhoA;
    for (int a = 0; a < 3; ++a) {
      acc[3] += (divB[a] - rhoB[a]) * (divB[a] - rhoB[a]);
      acc[4] += divB[a] * divB[a];
      acc[5] += rhoB[a] * rhoB[a];
    }
  }
  su2_block_partials<kSu2GaussAcc>(acc, A.partials);
}

__global__ __launch_bounds__(1024) void su2_gauss_finish_kernel(const double* partials, int nblocks, DevState* st) {
  __shared__ double red[16][kSu2GaussAcc];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double tot[kSu2GaussAcc] = {0, 0, 0, 0, 0, 0};
  for (int b = tid; b < nblocks; b += 1024)
    for (int k = 0; k < kSu2GaussAcc; ++k) tot[k] += partials[(size_t)b * kSu2GaussAcc + k];
  for (int k = 0; k < kSu2GaussAcc; ++k) {
    const double v = wsum64(tot[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  double S[kSu2GaussAcc] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < kSu2GaussAcc; ++k)
    for (int w = 0; w < 16; ++w) S[k] += red[w][k];
  const double dA = sqrt(S[1]) + sqrt(S[2]), dB = sqrt(S[4]) + sqrt(S[5]);
  st->obs.gauss = dA > 0.0 ? sqrt(S[0]) / dA : 0.0;
  st->obs.gauss_B = dB > 0.0 ? sqrt(S[3]) / dB : 0.0;
}

template <typename T>
static void su2_fill(lattice* h, Su2Args<T>& A, const PassDesc& pd) {
  for (int c = 0; c < kSu2Comp; ++c) {
    A.src[c] = static_cast<const T*>(h->buf[h->cur][c]);
    A.dst[c] = static_cast<T*>(h->buf[1 - h->cur][c]);
  }
  A.N = h->p.N;
  A.dx = h->dx;
  A.alpha = h->p.alpha;
  A.fmp2 = h->p.fstar_over_mp * h->p.fstar_over_mp;
  A.lam = h->p.lambda;
  A.m2 = h->p.m2[0];
  A.e = h->p.e;
  A.g = h->p.g;
  A.wf2 = h->p.omega_over_f * h->p.omega_over_f;
  A.h = h->p.dt;
  A.expand = h->p.expansion;
  A.fields_in_dst = 0;
  A.pd = pd;
  A.partials = h->partials;
  A.st = h->st;
}

// One pass of the shared schedule: drift (when wd != 0) into the other
// buffer, kick, finish; the buffers swap when the pass writes.
template <typename T>
static int su2_pass_t(lattice* h, const PassDesc& pd) {
  Su2Args<T> A;
  su2_fill(h, A, pd);
  const int64_t V = (int64_t)h->p.N * h->p.N * h->p.N;
  const int nb = (int)((V + 255) / 256);
  if (pd.wd != 0.0) {
    if (!pd.write) { set_error("SU(2) pass: a drift must write"); return LAT_EINVAL; }
    hipLaunchKernelGGL(su2_drift_kernel<T>, dim3(nb), dim3(256), 0, h->stream, A);
    CL_HIP(hipGetLastError());
    A.fields_in_dst = 1;
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (pd.write && 2 * h->timer_used + 1 < h->timer.size()) {
    ev0 = h->timer[2 * h->timer_used];
    ev1 = h->timer[2 * h->timer_used + 1];
    ++h->timer_used;
  }
  if (ev0) CL_HIP(hipEventRecord(ev0, h->stream));
  hipLaunchKernelGGL(su2_kick_kernel<T>, dim3(nb), dim3(256), 0, h->stream, A);
  CL_HIP(hipGetLastError());
  if (ev1) CL_HIP(hipEventRecord(ev1, h->stream));
  // the kick's nb records folded into R records in the second partials
  // buffer (it holds max_blocks >= R records of 16 sums), then the finish
  const int R = (int)std::min<int64_t>(kSu2FoldBlocks, h->max_blocks);
  hipLaunchKernelGGL(su2_fold_records<kSu2Acc>, dim3(R), dim3(256), 0, h->stream, A.partials, nb, h->partials2);
  CL_HIP(hipGetLastError());
  A.partials = h->partials2;
  hipLaunchKernelGGL(su2_finish_kernel<T>, dim3(1), dim3(kSu2FinishThreads), 0, h->stream, A, R);
  CL_HIP(hipGetLastError());
  if (pd.write) h->cur ^= 1;
  return LAT_OK;
}

template <typename T>
static int su2_gauss_t(lattice* h) {
  Su2Args<T> A;
  su2_fill(h, A, pass(0.0, 0.0, 0.0, MODE_VV, 0, 0));
  const int64_t V = (int64_t)h->p.N * h->p.N * h->p.N;
  const int nb = (int)((V + 255) / 256);
  hipLaunchKernelGGL(su2_gauss_kernel<T>, dim3(nb), dim3(256), 0, h->stream, A);
  CL_HIP(hipGetLastError());
  hipLaunchKernelGGL(su2_gauss_finish_kernel, dim3(1), dim3(1024), 0, h->stream, h->partials, nb, h->st);
  CL_HIP(hipGetLastError());
  return LAT_OK;
}

static int su2_pass(lattice* h, const PassDesc& pd) {
  return h->p.precision == LAT_FP32 ? su2_pass_t<float>(h, pd) : su2_pass_t<double>(h, pd);
}

int su2_step(lattice* h, int64_t n) {
  const std::vector<PassDesc> sched = pass_schedule(h->p.integrator, h->weights, &h->staggered, n);
  for (const PassDesc& pd : sched) {
    const int rc = su2_pass(h, pd);
    if (rc) return rc;
  }
  h->step += n;
  return LAT_OK;
}

int su2_energies(lattice* h) {
  int rc = h->p.precision == LAT_FP32 ? su2_gauss_t<float>(h) : su2_gauss_t<double>(h);
  if (rc) return rc;
  if (h->staggered) return su2_pass(h, pass(0.0, 0.0, 1.0, MODE_LF, 0, 0));
  return su2_pass(h, pass(0.0, 0.0, 0.0, MODE_VV, 0, 0));
}

// ---------------------------------------------------------------------------
// initial state (Sec. 7.2)
// ---------------------------------------------------------------------------
// Phi = (phi_0 + i phi_1, phi_2 + i phi_3)/sqrt 2 and pi = a^{3-alpha} Phi' from
// the FP64 real components; the charge densities rho_A, rho_B^a (Sec. 6.2 Gauss
// laws) as the real parts of four complex arrays.
template <typename T>
__global__ void su2_store_kernel(const double* f, const double* d, Su2Args<T> A, double2* rho, int64_t V,
                                 double cpi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const double is2 = 0.70710678118654752440084436210485;
  double ph[4], pq[4];
  for (int k = 0; k < 4; ++k) {
    ph[k] = f[(size_t)k * V + i] * is2;
    pq[k] = cpi * d[(size_t)k * V + i] * is2;
    A.dst[kPH + k][i] = (T)ph[k];
    A.dst[kPI + k][i] = (T)pq[k];
  }
  const Cx2<double> p0{ph[0], ph[1]}, p1{ph[2], ph[3]}, q0{pq[0], pq[1]}, q1{pq[2], pq[3]};
  const double cB = A.g / A.wf2;
  rho[i] = make_double2(2.0 * A.e / A.wf2 * (cross_im(p0, q0) + cross_im(p1, q1)), 0.0);
  rho[V + i] = make_double2(cB * (cross_im(p0, q1) + cross_im(p1, q0)), 0.0);
  rho[2 * V + i] = make_double2(cB * (-dot_re(p0, q1) + dot_re(p1, q0)), 0.0);
  rho[3 * V + i] = make_double2(cB * (cross_im(p0, q0) - cross_im(p1, q1)), 0.0);
}

template <typename T>
__global__ void su2_unit_links_kernel(Su2Args<T> A, int64_t V) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  for (int i = 0; i < 3; ++i) {
    A.dst[kTH + i][s] = T(0);
    A.dst[kUL + 4 * i][s] = T(1);
    A.dst[kUL + 4 * i + 1][s] = T(0);
    A.dst[kUL + 4 * i + 2][s] = T(0);
    A.dst[kUL + 4 * i + 3][s] = T(0);
  }
}

template <typename T>
static int su2_init_state_t(lattice* h) {
  const lattice_params& p = h->p;
  const int N = p.N;
  const int64_t V = (int64_t)N * N * N;
  const double a = p.a0, al = p.alpha, fmp2 = p.fstar_over_mp * p.fstar_over_mp;
  // every real component starts at phi0[0] (and dphi0[0]), as Sec. 7.2 does
  const double pb = p.phi0[0], db = p.dphi0[0];
  const double s = 4.0 * pb * pb, r2 = 0.5 * s;
  const double rho_hom = 4.0 * db * db / (2.0 * std::pow(a, 2.0 * al)) + p.lambda * r2 * r2 + p.m2[0] * r2;
  const double Hhom = p.expansion ? std::sqrt(fmp2 / 3.0 * std::pow(a, 2.0 * (al + 1.0)) * rho_hom) / a : 0.0;
  const double m2eff = p.lambda * (s + 2.0 * pb * pb) + p.m2[0];
  // scratch in the other state buffer: 8 V doubles of fields, then 4 V complex charges
  char* base = static_cast<char*>(h->buf[1 - h->cur][0]);
  double* fld = reinterpret_cast<double*>(base);
  double2* rho = reinterpret_cast<double2*>(base + (size_t)8 * V * sizeof(double));
  for (int n = 0; n < 4; ++n)
    for (int deriv = 0; deriv < 2; ++deriv) {
      int rc = charged_mode_field(h, n, deriv, m2eff, Hhom, deriv ? db : pb, fld + (size_t)(deriv * 4 + n) * V);
      if (rc) return rc;
    }
  Su2Args<T> A;
  su2_fill(h, A, pass(0.0, 0.0, 0.0, MODE_VV, 0, 0));
  for (int c = 0; c < kSu2Comp; ++c) A.dst[c] = static_cast<T*>(h->buf[h->cur][c]);
  const int thr = 256;
  const int blk = (int)((V + thr - 1) / thr);
  hipLaunchKernelGGL(su2_store_kernel<T>, dim3(blk), dim3(thr), 0, h->stream, fld, fld + 4 * V, A, rho, V,
                     std::pow(a, 3.0 - al));
  CL_HIP(hipGetLastError());
  hipLaunchKernelGGL(su2_unit_links_kernel<T>, dim3(blk), dim3(thr), 0, h->stream, A, V);
  CL_HIP(hipGetLastError());
  // each charge: forward DFT into its own slot, then the three minimum-norm solutions
  double2* F = reinterpret_cast<double2*>(h->fft);
  for (int q = 0; q < 4; ++q) {
    CL_HIP(hipMemcpyAsync(F, rho + (size_t)q * V, (size_t)V * sizeof(double2), hipMemcpyDeviceToDevice, h->stream));
    int rc = run_fft3d(h, +1, 1.0);
    if (rc) return rc;
    CL_HIP(hipMemcpyAsync(rho + (size_t)q * V, F, (size_t)V * sizeof(double2), hipMemcpyDeviceToDevice, h->stream));
  }
  for (int q = 0; q < 4; ++q) {
    void* out[3];
    for (int i = 0; i < 3; ++i) out[i] = q == 0 ? h->buf[h->cur][kPA + i] : h->buf[h->cur][kPB + 3 * i + (q - 1)];
    int rc = gauss_solve_fields(h, rho + (size_t)q * V, out, p.precision == LAT_FP32);
    if (rc) return rc;
  }
  int rc = upload_scalars(h, a, 0.0, 0.0);
  if (rc) return rc;
  h->staggered = 0;
  h->step = 0;
  if (p.expansion) {
    rc = su2_energies(h);
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

int su2_init_state(lattice* h) {
  return h->p.precision == LAT_FP32 ? su2_init_state_t<float>(h) : su2_init_state_t<double>(h);
}

}  // namespace cl
