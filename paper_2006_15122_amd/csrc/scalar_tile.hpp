// Device code of the fused scalar pass, shared by the single-lattice and the
// batched launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "common.hpp"

namespace cl {

template <typename T>
struct ScalarArgs {
  const T* src[4];   // phi_0, phi_1, pi_0, pi_1 (nf = 1 uses entries 0 and 2)
  T* dst[4];
  int N;
  int XC;            // x-planes per block
  int swizzle;       // map consecutive blocks of one XCD to neighbouring tiles
  double dx, alpha, fmp2, m2_0, m2_1, lam, q, h;
  int expand;
  PassDesc pd;
  double* partials;  // [gridDim.x][NACC]
  DevState* st;
  PrevPass prev;     // single-lattice passes only; batched launches leave it empty
};

// Field loads and stores through global-address-space pointers.  The batched
// pass takes its field pointers from a table in device memory, where the
// compiler cannot tell they address global memory; it would emit flat
// accesses, which count against the LDS wait counter as well, so that every
// wait for the stencil's LDS reads would also wait for the prefetched planes.
template <typename T>
__device__ __forceinline__ T load_g(const T* base, size_t o) {
  return ((const __attribute__((address_space(1))) T*)base)[o];
}
template <typename T>
__device__ __forceinline__ void store_g_nt(T v, T* base, size_t o) {
  __builtin_nontemporal_store(v, &((__attribute__((address_space(1))) T*)base)[o]);
}

// Accumulators of one pass.  FULL (observation passes): per field
// <pi_in^2>, <pi_E^2>, <grad^2>, <phi>, <phi^2>, then the three potential
// terms.  Stepping passes keep only what the scale-factor kernel needs:
// sum_f <pi_in^2>, sum_f <pi_E^2>, sum_f <grad^2>, <V>.
template <int NF, bool FULL>
struct Acc {
  static constexpr int N = FULL ? 5 * NF + 3 : 4;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// dV/dphi_f with the couplings as hi + lo pairs (no coherent rounding of them)
template <typename T, int NF>
__device__ __forceinline__ T dpot(int f, const T (&p)[NF], const Coef<T>& m2_0, const Coef<T>& m2_1,
                                  const Coef<T>& lam, const Coef<T>& q) {
  if (f == 0) {
    T d = fma_c(lam, p[0] * p[0] * p[0], mul_c(m2_0, p[0]));
    if constexpr (NF > 1) d = fma_c(q, p[1] * p[1] * p[0], d);
    return d;
  } else {
    if constexpr (NF > 1) return fma_c(q, p[0] * p[0] * p[1], mul_c(m2_1, p[1]));
    return T(0);
  }
}

// Reduce the per-thread accumulators of a block into partials[blockIdx.x]
// (wave shuffles, then the waves in order).  No fence or atomic here: the
// cross-block combination happens in scalar_finish_kernel, after the kernel
// boundary has made every block's partials visible to every XCD.
template <typename T, int NF, bool FULL, int NT>
__device__ void block_partials(const ScalarArgs<T>& A, double (&acc)[Acc<NF, FULL>::N], int pidx) {
  constexpr int NACC = Acc<NF, FULL>::N;
  constexpr int NW = NT / 64;
  __shared__ double red[NW][NACC];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (tid < NACC) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w][tid];
    A.partials[(size_t)pidx * NACC + tid] = s;
  }
}

// One block: combine the partials of all nblocks blocks in block order
// (thread t takes blocks t, t+256, ...; then shuffles and waves in order),
// form the volume averages (Sec. 4.3.2/4.4) and advance b in FP64,
//   b_out = b_in + (wk1 + wk2) h K_a(a', E),
//   K_a = (1/3)(f*/m_p)^2 a'^{1+2 alpha}[(alpha-2)E_K + alpha E_G + (alpha+1)E_V].
// Sum NB consecutive partial records (starting at `first`) in a fixed order
// with one block of NT threads; thread 0 returns the totals in S.
template <int NACC, int NT>
__device__ bool reduce_partials(const double* partials, int first, int nb, double (&S)[NACC]) {
  constexpr int NW = NT / 64;
  __shared__ double red[NW][NACC];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double tot[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) tot[k] = 0.0;
  for (int b = tid; b < nb; b += NT) {
#pragma unroll
    for (int k = 0; k < NACC; ++k) tot[k] += partials[(size_t)(first + b) * NACC + k];
  }
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    const double s = wave_sum(tot[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (tid != 0) return false;
  for (int k = 0; k < NACC; ++k) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w][k];
    S[k] = s;
  }
  return true;
}

// From the lattice sums S of pass `pd`, which started from state `in`: the
// volume averages (Sec. 4.3.2/4.4) and the FP64 advance of b,
//   b_out = b_in + (wk1 + wk2) h K_a(a', E),
//   K_a = (1/3)(f*/m_p)^2 a'^{1+2 alpha}[(alpha-2)E_K + alpha E_G + (alpha+1)E_V].
// The resulting state goes to `out` (may be `in`; nullptr: not stored); a and b
// after the pass are returned in a_next, b_next.
template <typename T, int NF, bool FULL>
__device__ void finish_state(const ScalarArgs<T>& A, const PassDesc& pd, const DevState* in,
                             const double (&S)[Acc<NF, FULL>::N], DevState* out, double& a_next,
                             double& b_next) {
  constexpr int NACC = Acc<NF, FULL>::N;
  const double a_in = in->a, b_in = in->b, eta_in = in->eta;
  const double anew = A.expand ? a_in + pd.wd * A.h * b_in : a_in;
  const double V = (double)A.N * (double)A.N * (double)A.N;
  const double al = A.alpha;
  const double a2 = anew * anew, a6 = a2 * a2 * a2, dx2 = A.dx * A.dx;
  lattice_obs o;
  o.EK = o.EG = 0.0;
  o.EK_f[0] = o.EK_f[1] = o.EG_f[0] = o.EG_f[1] = 0.0;
  o.mean_f[0] = o.mean_f[1] = o.meansq_f[0] = o.meansq_f[1] = 0.0;
  bool bad = false;
  if constexpr (FULL) {
    for (int f = 0; f < NF; ++f) {
      const double k1 = S[5 * f + 0] / V, k2 = S[5 * f + 1] / V;
      const double ek = (pd.mode == MODE_LF) ? (k1 + k2) / (4.0 * a6) : k2 / (2.0 * a6);
      const double eg = S[5 * f + 2] / V / (2.0 * a2 * dx2);
      o.EK_f[f] = ek;
      o.EG_f[f] = eg;
      o.mean_f[f] = S[5 * f + 3] / V;
      o.meansq_f[f] = S[5 * f + 4] / V;
      o.EK += ek;
      o.EG += eg;
    }
    o.EV_term[0] = S[5 * NF + 0] / V;
    o.EV_term[1] = S[5 * NF + 1] / V;
    o.EV_term[2] = S[5 * NF + 2] / V;
    o.EV = o.EV_term[0] + o.EV_term[1] + o.EV_term[2];
  } else {
    const double k1 = S[0] / V, k2 = S[1] / V;
    o.EK = (pd.mode == MODE_LF) ? (k1 + k2) / (4.0 * a6) : k2 / (2.0 * a6);
    o.EG = S[2] / V / (2.0 * a2 * dx2);
    o.EV = S[3] / V;
    o.EV_term[0] = o.EV_term[1] = o.EV_term[2] = NAN;
    for (int f = 0; f < 2; ++f) o.EK_f[f] = o.EG_f[f] = o.mean_f[f] = o.meansq_f[f] = NAN;
  }
  for (int k = 0; k < NACC; ++k) bad = bad || !isfinite(S[k]);
  const double rho = o.EK + o.EG + o.EV;
  double b_out = b_in, b_sync = b_in, hc = 0.0;
  if (A.expand) {
    const double Ka = A.fmp2 / 3.0 * apow(anew, 1.0 + 2.0 * al) *
                      ((al - 2.0) * o.EK + al * o.EG + (al + 1.0) * o.EV);
    b_out = b_in + (pd.wk1 + pd.wk2) * A.h * Ka;
    b_sync = (pd.mode == MODE_LF) ? 0.5 * (b_in + b_out) : b_in + pd.wk1 * A.h * Ka;
    const double rhs = A.fmp2 / 3.0 * apow(anew, 2.0 * (al + 1.0)) * rho;
    hc = fabs(b_sync * b_sync - rhs) / (b_sync * b_sync);
  }
  const double eta_new = eta_in + pd.wd * A.h;
  o.eta = eta_new;
  o.a = anew;
  o.b = b_sync;
  o.H = b_sync / anew;
  o.EK_A = o.EG_A = 0.0;
  o.rho = rho;
  o.p = o.EK - o.EG / 3.0 - o.EV;
  o.w = rho != 0.0 ? o.p / rho : 0.0;
  o.hc = hc;
  o.gauss = NAN;
  o.step = 0;
  o.staggered = (pd.mode == MODE_LF) ? 1 : 0;
  o.reserved = 0;
  a_next = pd.update ? anew : a_in;
  b_next = pd.update ? b_out : b_in;
  if (!out) return;
  if (out != in) *out = *in;
  out->obs = o;
  if (bad) out->nonfinite = 1;
  if (pd.update) {
    out->a = anew;
    out->b = b_out;
    out->eta = eta_new;
  }
}

// In-place finish of the pass described by A (the batched path).
template <typename T, int NF, bool FULL>
__device__ void finish_from_sums(const ScalarArgs<T>& A, const double (&S)[Acc<NF, FULL>::N]) {
  double an, bn;
  finish_state<T, NF, FULL>(A, A.pd, A.st, S, A.st, an, bn);
}

// One block: combine the partials of all nblocks tiles in block order and
// update the homogeneous state.
// One block of kFinishThreads threads: four waves leave each thread the
// registers for its FP64 sums (1024 threads, held to 128 VGPRs, spilled them).
constexpr int kFinishThreads = 256;

template <typename T, int NF, bool FULL>
__global__ __launch_bounds__(kFinishThreads) void scalar_finish_kernel(ScalarArgs<T> A, int nblocks, DevState* out) {
  double S[Acc<NF, FULL>::N];
  if (!reduce_partials<Acc<NF, FULL>::N, kFinishThreads>(A.partials, 0, nblocks, S)) return;
  double an, bn;
  finish_state<T, NF, FULL>(A, A.pd, A.st, S, out, an, bn);
}

// One tile (index `tile` in the order z-tile fastest, then y-tile, then
// x-chunk) of one lattice; its sums go to partial record `pidx`.  get_ab(a, b)
// supplies the scale factor and its derivative at the start of the pass; it
// is called once the first planes' loads are in flight (it may reduce the
// previous pass's records and synchronise the block).
template <typename T, int NF, bool FULL, int TZ, int BY, int RY, typename GetAB>
__device__ __forceinline__ void scalar_tile(const ScalarArgs<T>& A, int tile, int pidx, GetAB get_ab) {
  constexpr int TY = BY * RY;
  constexpr int NT = TZ * BY;
  constexpr int LZ = TZ + 2;
  constexpr int NACC = Acc<NF, FULL>::N;
  __shared__ T lds[NF][TY + 2][LZ];

  const int N = A.N;
  const int tid = threadIdx.x;
  const int tz = tid % TZ, ty = tid / TZ;
  const int nzt = N / TZ, nyt = N / TY;
  int bid = tile;
  const int zt = bid % nzt;
  bid /= nzt;
  const int yt = bid % nyt;
  const int xcI = bid / nyt;
  const int z0 = zt * TZ, y0 = yt * TY, x0 = xcI * A.XC;
  const size_t NN = (size_t)N * N;

  const Coef<T> ckick = ucoef<T>((A.pd.wk1 + A.pd.wk2) * A.h);
  const Coef<T> cE = ucoef<T>((A.pd.mode == MODE_LF ? (A.pd.wk1 + A.pd.wk2) : A.pd.wk1) * A.h);
  const T m2_0 = (T)A.m2_0, m2_1 = (T)A.m2_1, lam = (T)A.lam, q = (T)A.q;
  const Coef<T> m2_0c = ucoef<T>(A.m2_0), m2_1c = ucoef<T>(A.m2_1), lamc = ucoef<T>(A.lam), qc_ = ucoef<T>(A.q);
  const T half = T(0.5), quarter = T(0.25);
  const bool lf = A.pd.mode == MODE_LF;

  double acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = 0.0;

  const int z = z0 + tz;
  // register planes: pm = drifted x-1, pc = drifted x, (pn, qn) = raw x+1,
  // (pf, qf) = raw x+2 in flight; qc = momentum at x
  T pm[NF][RY], pc[NF][RY], qc[NF][RY], pn[NF][RY], qn[NF][RY], pf[NF][RY], qf[NF][RY];

  // halo item owned by this thread (at most one: 2 TZ + 2 TY <= NT)
  constexpr int NH = 2 * TZ + 2 * TY;
  static_assert(NH <= NT, "halo larger than block");
  int hy = 0, hz = 0, hly = 0, hlz = 0;
  const bool has_halo = tid < NH;
  if (has_halo) {
    if (tid < TZ) { hly = 0; hlz = 1 + tid; hy = (y0 - 1 + N) % N; hz = z0 + tid; }
    else if (tid < 2 * TZ) { hly = TY + 1; hlz = 1 + tid - TZ; hy = (y0 + TY) % N; hz = z0 + tid - TZ; }
    else if (tid < 2 * TZ + TY) { hly = 1 + tid - 2 * TZ; hlz = 0; hy = y0 + tid - 2 * TZ; hz = (z0 - 1 + N) % N; }
    else { hly = 1 + tid - 2 * TZ - TY; hlz = TZ + 1; hy = y0 + tid - 2 * TZ - TY; hz = (z0 + TZ) % N; }
  }
  T hp1[NF], hq1[NF], hp2[NF], hq2[NF];

  auto row_off = [&](int x, int y) -> size_t { return (size_t)x * NN + (size_t)y * N; };

  // raw phi and pi of the own columns of plane x
  auto load_own = [&](int x, T (&p)[NF][RY], T (&pq)[NF][RY]) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const size_t o = row_off(x, y0 + r * BY + ty) + z;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        p[f][r] = load_g(A.src[f], o);
        pq[f][r] = load_g(A.src[2 + f], o);
      }
    }
  };
  auto load_halo = [&](int x, T (&p)[NF], T (&pq)[NF]) {
    if (has_halo) {
      const size_t o = row_off(x, hy) + hz;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        p[f] = load_g(A.src[f], o);
        pq[f] = load_g(A.src[2 + f], o);
      }
    }
  };

  // prologue: planes x0-1 (drifted), x0 (drifted, into LDS), x0+1 (raw, in flight)
  const int xm = (x0 - 1 + N) % N;
  load_own(xm, pm, qf);  // qf: momentum of plane x0-1, only needed for its drift

  // homogeneous coefficients (FP64, identical in every block), while the
  // loads above are in flight
  double a_in, b_in;
  get_ab(a_in, b_in);
  load_own(x0, pc, qc);
  load_halo(x0, hp1, hq1);
  load_own((x0 + 1) % N, pn, qn);
  if (A.XC > 1) load_halo((x0 + 1) % N, hp2, hq2);
  const double anew = A.expand ? a_in + A.pd.wd * A.h * b_in : a_in;
  const double amid = 0.5 * (a_in + anew);
  const Coef<T> cdrift = ucoef<T>(A.pd.wd * A.h * apow(amid, -(3.0 - A.alpha)));
  const Coef<T> clap = ucoef<T>(apow(anew, 1.0 + A.alpha) / (A.dx * A.dx));
  const Coef<T> cpot = ucoef<T>(apow(anew, 3.0 + A.alpha));
  // drifted plane into LDS: own columns from registers, halo drifted here
  auto store_lds = [&](const T (&p)[NF][RY], const T (&hp)[NF], const T (&hq)[NF]) {
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
      for (int f = 0; f < NF; ++f) lds[f][1 + r * BY + ty][1 + tz] = p[f][r];
    if (has_halo) {
#pragma unroll
      for (int f = 0; f < NF; ++f) lds[f][hly][hlz] = fma_c(cdrift, hq[f], hp[f]);
    }
  };
  {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        pm[f][r] = fma_c(cdrift, qf[f][r], pm[f][r]);
        pc[f][r] = fma_c(cdrift, qc[f][r], pc[f][r]);
      }
    store_lds(pc, hp1, hq1);
  }

  // One plane of the stencil.  (pn, qn) hold raw plane x+1 and (hpa, hqa) the
  // halo of x+1; plane x+2 is loaded into (pf, qf) and (hpb, hqb).  The loop
  // below calls this twice per trip with the two register sets swapped, so
  // that no register copy has to wait for the loads just issued: they are
  // first used one plane later.
  auto plane = [&](int i, T (&pn)[NF][RY], T (&qn)[NF][RY], T (&pf)[NF][RY], T (&qf)[NF][RY],
                   T (&hpa)[NF], T (&hqa)[NF], T (&hpb)[NF], T (&hqb)[NF]) {
    const int x = x0 + i;
    // issue loads of plane x+2, two planes ahead of the stencil
    if (i + 1 < A.XC) {
      load_own((x + 2) % N, pf, qf);
      if (i + 2 < A.XC) load_halo((x + 2) % N, hpb, hqb);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ly = 1 + r * BY + ty;
      T cur[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) cur[f] = pc[f][r];
      const size_t o = row_off(x, y0 + r * BY + ty) + z;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const T pnext = fma_c(cdrift, qn[f][r], pn[f][r]);
        const T yp = lds[f][ly + 1][1 + tz], ym = lds[f][ly - 1][1 + tz];
        const T zp = lds[f][ly][2 + tz], zm = lds[f][ly][tz];
        // differences first: each neighbour minus the site is exact in
        // storage precision for nearby values, so the Laplacian of the small
        // fluctuations does not cancel against the condensate
        const T c = cur[f];
        const T lap = ((pm[f][r] - c) + (pnext - c)) + ((yp - c) + (ym - c)) + ((zp - c) + (zm - c));
        const T K = fma_c(clap, lap, -mul_c(cpot, dpot<T, NF>(f, cur, m2_0c, m2_1c, lamc, qc_)));
        const T pin = qc[f][r];
        const T pout = fma_c(ckick, K, pin);
        const T pe = fma_c(cE, K, pin);
        if constexpr (!FULL) {
          // stepping passes always store and observation passes never do (the
          // launcher checks pd.write against this), so no branch splits the
          // count of memory operations in flight.  Streaming stores: the new
          // state is read again only by the next pass, so keep it from
          // evicting the halo rows other tiles still need
          store_g_nt(cur[f], A.dst[f], o);
          store_g_nt(pout, A.dst[2 + f], o);
        }
        const T gx = pnext - cur[f], gy = yp - cur[f], gz = zp - cur[f];
        if constexpr (FULL) {
          acc[5 * f + 0] += (double)(pin * pin);
          acc[5 * f + 1] += (double)(pe * pe);
          acc[5 * f + 2] += (double)(gx * gx + gy * gy + gz * gz);
          acc[5 * f + 3] += (double)cur[f];
          acc[5 * f + 4] += (double)(cur[f] * cur[f]);
        } else {
          if (lf) acc[0] += (double)(pin * pin);
          acc[1] += (double)(pe * pe);
          acc[2] += (double)(gx * gx + gy * gy + gz * gz);
        }
      }
      const T p2 = cur[0] * cur[0];
      if constexpr (FULL) {
        if constexpr (NF > 1) {
          const T c2 = cur[1] * cur[1];
          acc[5 * NF + 0] += (double)(half * (m2_0 * p2 + m2_1 * c2));
          acc[5 * NF + 2] += (double)(half * q * p2 * c2);
        } else {
          acc[5 * NF + 0] += (double)(half * m2_0 * p2);
        }
        acc[5 * NF + 1] += (double)(quarter * lam * p2 * p2);
      } else {
        T v = half * m2_0 * p2 + quarter * lam * p2 * p2;
        if constexpr (NF > 1) {
          const T c2 = cur[1] * cur[1];
          v += half * (m2_1 * c2 + q * p2 * c2);
        }
        acc[3] += (double)v;
      }
    }
    __syncthreads();
    // shift: plane x+1 becomes current (x+2 becomes next by the swap)
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        pm[f][r] = pc[f][r];
        pc[f][r] = fma_c(cdrift, qn[f][r], pn[f][r]);
        qc[f][r] = qn[f][r];
      }
    if (i + 1 < A.XC) store_lds(pc, hpa, hqa);
  };
  for (int i = 0; i < A.XC; i += 2) {
    plane(i, pn, qn, pf, qf, hp2, hq2, hp1, hq1);
    if (i + 1 < A.XC) plane(i + 1, pf, qf, pn, qn, hp1, hq1, hp2, hq2);
  }
  block_partials<T, NF, FULL, NT>(A, acc, pidx);
}

// Up to four rows per thread the kernel is held to four waves per SIMD (128
// VGPRs): the first plane's loads in flight across the chained finish would
// otherwise push it past that and halve the blocks per CU.
template <typename T, int NF, bool FULL, int TZ, int BY, int RY>
__global__ __launch_bounds__(TZ* BY, RY <= 4 ? 4 : 1) void scalar_pass_kernel(ScalarArgs<T> A) {
  int bid = blockIdx.x;
  if (A.swizzle) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  auto get_ab = [&](double& a_in, double& b_in) {
    if (A.prev.partials) {
      // finish of the previous pass (stepping passes only, Acc<NF, false>)
      constexpr int NP = Acc<NF, false>::N;
      __shared__ double ab[2];
      double S[NP];
      if (reduce_partials<NP, TZ * BY>(A.prev.partials, 0, A.prev.nblocks, S)) {
        double an, bn;
        finish_state<T, NF, false>(A, A.prev.pd, A.st, S, blockIdx.x == 0 ? A.prev.out : nullptr, an, bn);
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
  };
  scalar_tile<T, NF, FULL, TZ, BY, RY>(A, bid, blockIdx.x, get_ab);
}


}  // namespace cl
