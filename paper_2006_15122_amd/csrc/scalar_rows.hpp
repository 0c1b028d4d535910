// Full-row tile of the fused scalar pass (stepping passes).
//
// A block holds whole z-rows of the lattice: N = W NL sites per row, W
// consecutive sites per lane moved as one 16-byte access (W = 4 in FP32
// storage, 2 in FP64).  It owns BY consecutive y-rows and marches along x
// over XC planes like the general tile, with each site's drift and kick
// written term for term as there: from the same a and b, a pass gives every
// site the general tile's new field and momentum bit for bit.  The energy
// terms of a lane's W sites are summed in storage precision before they join
// the FP64 totals, so the sums (and with them a and b after the pass) agree
// with the general tile's to rounding, not bit for bit.  What changes is the
// memory side: the periodic z-neighbours of a row are in the row itself (no
// z halo loads at all), every global access is a whole 16-byte lane segment
// of a row, and one address serves W sites.  The only halo left is the two
// y-rows above and below the block, spread over all lanes.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"
#include "scalar_tile.hpp"

namespace cl {

// W consecutive sites of one row: the vector a lane loads and stores
template <typename T, int W>
struct RowVec {
  typedef T type __attribute__((ext_vector_type(W)));
};

__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }

// the W sites' terms of one lane, summed pairwise
template <typename T, int W>
__device__ __forceinline__ T lane_sum(const T (&v)[W]) {
  if constexpr (W == 4) return (v[0] + v[1]) + (v[2] + v[3]);
  if constexpr (W == 2) return v[0] + v[1];
  return v[0];
}

template <typename T, int W, int NF, int NL, int BY, typename GetAB>
__device__ __forceinline__ void scalar_rows(const ScalarArgs<T>& A, int tile, int pidx, GetAB get_ab) {
  using VW = typename RowVec<T, W>::type;  // W consecutive sites
  constexpr int N = W * NL;
  constexpr int NT = NL * BY;
  constexpr int NACC = Acc<NF, false>::N;
  static_assert(NT % 64 == 0 && NT <= 1024, "block of whole waves");
  // drifted planes in two buffers: plane x0 + i in buffer i & 1 (x0 - 1 in
  // buffer 1), rows y0-1 .. y0+BY, each a whole z-row; the x-1 neighbours of
  // the stencil are read from the other buffer
  __shared__ VW lds[2][NF][BY + 2][NL];

  const int tid = threadIdx.x;
  const int tz = tid % NL, ty = tid / NL;
  constexpr int nyt = N / BY;
  const int yt = tile % nyt, xcI = tile / nyt;
  const int y0 = yt * BY, x0 = xcI * A.XC;
  const size_t NN = (size_t)N * N;

  const Coef<T> ckick = ucoef<T>((A.pd.wk1 + A.pd.wk2) * A.h);
  const Coef<T> cE = ucoef<T>((A.pd.mode == MODE_LF ? (A.pd.wk1 + A.pd.wk2) : A.pd.wk1) * A.h);
  const Coef<T> m2_0c = ucoef<T>(A.m2_0), m2_1c = ucoef<T>(A.m2_1), lamc = ucoef<T>(A.lam), qc_ = ucoef<T>(A.q);
  // potential-energy density V = p2 (m2_0/2 + lam p2/4) + c2 (m2_1/2 + q p2/2)
  const T hm2_0 = (T)(0.5 * A.m2_0), qlam = (T)(0.25 * A.lam), hm2_1 = (T)(0.5 * A.m2_1), hqq = (T)(0.5 * A.q);
  const bool lf = A.pd.mode == MODE_LF;

  double acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = 0.0;

  const int y = y0 + ty;
  const int ly = 1 + ty;
  // register planes (four sites each): pc = drifted x, qc = momentum at x,
  // (pn, qn) = raw x+1, (pf, qf) = raw x+2 in flight
  VW pc[NF], qc[NF], pn[NF], qn[NF], pf[NF], qf[NF];

  // halo rows y0-1 and y0+BY of plane x+1, loaded one plane ahead of their
  // use: 2 NF N single sites spread over all lanes, KH per lane
  constexpr int NHI = 2 * NF * N;
  constexpr int KH = (NHI + NT - 1) / NT;
  T hp[KH], hq[KH];

  auto at = [&](const T* base, size_t o) { return *reinterpret_cast<const VW*>(base + o); };
  auto load_own = [&](int x, VW (&p)[NF], VW (&pq)[NF]) {
    const size_t o = (size_t)x * NN + (size_t)y * N + W * tz;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      p[f] = at(A.src[f], o);
      pq[f] = at(A.src[2 + f], o);
    }
  };
  // halo item k of this lane: row r (0: y0-1, 1: y0+BY), field f, site z
  auto halo_item = [&](int k, int& r, int& f, int& z) {
    const int it = tid + k * NT;
    r = it / (NF * N);
    f = (it / N) % NF;
    z = it % N;
    return it < NHI;
  };
  auto load_halo = [&](int x) {
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      int r, f, z;
      if (halo_item(k, r, f, z)) {
        const int yy = r == 0 ? (y0 - 1 + N) % N : (y0 + BY) % N;
        const size_t o = (size_t)x * NN + (size_t)yy * N + z;
        hp[k] = (f == 0 ? A.src[0] : A.src[NF - 1])[o];
        hq[k] = (f == 0 ? A.src[2] : A.src[2 + NF - 1])[o];
      }
    }
  };

  // prologue: planes x0-1 (drifted, into buffer 1), x0 (drifted, into
  // buffer 0 with its halo), x0+1 (raw, in flight)
  const int xm = (x0 - 1 + N) % N;
  VW pm[NF];
  load_own(xm, pm, qf);  // qf: momentum of plane x0-1, only needed for its drift
  double a_in, b_in;
  get_ab(a_in, b_in);
  load_own(x0, pc, qc);
  load_halo(x0);
  load_own((x0 + 1) % N, pn, qn);
  const double anew = A.expand ? a_in + A.pd.wd * A.h * b_in : a_in;
  const double amid = 0.5 * (a_in + anew);
  const Coef<T> cdrift = ucoef<T>(A.pd.wd * A.h * apow(amid, -(3.0 - A.alpha)));
  const Coef<T> clap = ucoef<T>(apow(anew, 1.0 + A.alpha) / (A.dx * A.dx));
  const Coef<T> cpot = ucoef<T>(apow(anew, 3.0 + A.alpha));
  auto drift = [&](const VW& qv, const VW& pv) {
    VW r;
#pragma unroll
    for (int e = 0; e < W; ++e) r[e] = fma_c(cdrift, qv[e], pv[e]);
    return r;
  };
  // the drifted plane into LDS buffer b: own rows from registers, halo rows
  // drifted here
  auto store_lds = [&](int b) {
#pragma unroll
    for (int f = 0; f < NF; ++f) lds[b][f][ly][tz] = pc[f];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      int r, f, z;
      if (halo_item(k, r, f, z)) {
        T* row = reinterpret_cast<T*>(&lds[b][f][r == 0 ? 0 : BY + 1][0]);
        row[z] = fma_c(cdrift, hq[k], hp[k]);
      }
    }
  };
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    lds[1][f][ly][tz] = drift(qf[f], pm[f]);
    pc[f] = drift(qc[f], pc[f]);
  }
  store_lds(0);

  // One plane (x = x0 + i, in buffer B = i & 1); called twice per trip with
  // the register sets swapped (see the general tile): (pn, qn) hold raw plane
  // x+1, plane x+2 is loaded into (pf, qf), the halo rows of x+1 into (hp, hq).
  auto plane = [&](int i, auto bsel, VW (&pn)[NF], VW (&qn)[NF], VW (&pf)[NF], VW (&qf)[NF]) {
    constexpr int B = decltype(bsel)::value;
    const int x = x0 + i;
    if (i + 1 < A.XC) {
      load_own((x + 2) % N, pf, qf);
      load_halo((x + 1) % N);
    }
    __syncthreads();
    const size_t o = (size_t)x * NN + (size_t)y * N + W * tz;
    // plane x+1 drifted, in place
#pragma unroll
    for (int f = 0; f < NF; ++f) pn[f] = drift(qn[f], pn[f]);
    // the potential at the lane's W sites, summed pairwise in storage
    // precision and added to the FP64 total once per plane
    {
      T v4[W];
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const T p2 = pc[0][e] * pc[0][e];
        T v = p2 * fma_t(qlam, p2, hm2_0);
        if constexpr (NF > 1) {
          const T c2 = pc[1][e] * pc[1][e];
          v = fma_t(c2, fma_t(hqq, p2, hm2_1), v);
        }
        v4[e] = v;
      }
      acc[3] += (double)lane_sum<T, W>(v4);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const VW xm4 = lds[1 - B][f][ly][tz];
      const VW yp = lds[B][f][ly + 1][tz], ym = lds[B][f][ly - 1][tz];
      // the z-neighbours outside the lane's four sites, periodic in the row
      const T zlo = lds[B][f][ly][(tz + NL - 1) % NL][W - 1];
      const T zhi = lds[B][f][ly][(tz + 1) % NL][0];
      VW pout;
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int e = 0; e < W; ++e) {
        T cur[NF];
#pragma unroll
        for (int g = 0; g < NF; ++g) cur[g] = pc[g][e];
        const T c = cur[f];
        const T zp = e == W - 1 ? zhi : pc[f][e + 1];
        const T zm = e == 0 ? zlo : pc[f][e - 1];
        // the general tile's Laplacian, term for term
        const T lap = ((xm4[e] - c) + (pn[f][e] - c)) + ((yp[e] - c) + (ym[e] - c)) + ((zp - c) + (zm - c));
        const T K = fma_c(clap, lap, -mul_c(cpot, dpot<T, NF>(f, cur, m2_0c, m2_1c, lamc, qc_)));
        const T pin = qc[f][e];
        pout[e] = fma_c(ckick, K, pin);
        const T pe = fma_c(cE, K, pin);
        const T gx = pn[f][e] - c, gy = yp[e] - c, gz = zp - c;
        s0 = fma_t(pin, pin, s0);
        s1 = fma_t(pe, pe, s1);
        s2 += gx * gx + gy * gy + gz * gz;
      }
      // the W sites' terms summed in storage precision, then into the FP64 totals
      if (lf) acc[0] += (double)s0;
      acc[1] += (double)s1;
      acc[2] += (double)s2;
      // streaming stores of the new state (read again only by the next pass)
      __builtin_nontemporal_store(pc[f], reinterpret_cast<VW*>(A.dst[f] + o));
      __builtin_nontemporal_store(pout, reinterpret_cast<VW*>(A.dst[2 + f] + o));
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      pc[f] = pn[f];
      qc[f] = qn[f];
    }
    // plane x+1 into the buffer of x-1, which no lane reads any more
    if (i + 1 < A.XC) store_lds(1 - B);
  };
  for (int i = 0; i < A.XC; i += 2) {
    plane(i, std::integral_constant<int, 0>{}, pn, qn, pf, qf);
    if (i + 1 < A.XC) plane(i + 1, std::integral_constant<int, 1>{}, pf, qf, pn, qn);
  }
  block_partials<T, NF, false, NT>(A, acc, pidx);
}

// About 145 VGPRs: one 512-lane block per CU.  Holding it to 128 (two
// blocks per CU) spills inside the plane loop and is slower.
template <typename T, int W, int NF, int NL, int BY>
__global__ __launch_bounds__(NL* BY) void scalar_rows_kernel(ScalarArgs<T> A) {
  int bid = blockIdx.x;
  if (A.swizzle) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  auto get_ab = [&](double& a_in, double& b_in) {
    if (A.prev.partials) {
      constexpr int NP = Acc<NF, false>::N;
      __shared__ double ab[2];
      double S[NP];
      if (reduce_partials<NP, NL * BY>(A.prev.partials, 0, A.prev.nblocks, S)) {
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
  scalar_rows<T, W, NF, NL, BY>(A, bid, blockIdx.x, get_ab);
}

}  // namespace cl
