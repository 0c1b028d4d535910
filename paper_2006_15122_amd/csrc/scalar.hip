// Fused scalar-field pass for gfx950: drift, 7-point stencil kick, FP64
// volume averages and the scale-factor update, in one sweep over the lattice.
//
// Method (arXiv:2006.15122): Hamiltonian form of the scalar EOM (Sec. 4.2.3)
//   phi' = a^{-(3-alpha)} pi,  pi' = a^{1+alpha} lap phi - a^{3+alpha} V_{,phi},
//   b'   = (1/3)(f*/m_p)^2 a^{1+2 alpha}[(alpha-2) E_K + alpha E_G + (alpha+1) E_V],
// integrated by velocity Verlet / Yoshida (Sec. 4.2.3, 4.3.2) or staggered leapfrog
// scheme III (Sec. 4.2.1).  Consecutive kicks of the Verlet chain are merged
// (Sec. 3.3.2: velocity Verlet is leapfrog plus a synchronising half kick), so
// one pass = drift of sub-step p followed by the kick that closes p and opens
// p+1.  The drift needs the global energies of the previous pass: a one-block
// finish kernel reduces the per-tile FP64 partials in a fixed order and
// advances a and b in FP64 before the next pass starts.
//
// Tiling: a block owns a TY x TZ tile of the (y, z) plane and marches along x
// over XC planes.  z is the fastest index, so each wavefront loads contiguous
// rows.  The drifted plane x (with a one-site y/z halo) sits in LDS; the x-1,
// x+1 neighbours stay in registers.  Halo sites are drifted redundantly by the
// neighbouring tiles, which removes a separate drift pass over HBM.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "scalar_rows.hpp"
#include "scalar_tile.hpp"

namespace cl {

// ---------------------------------------------------------------------------
// Host-side launch table
// ---------------------------------------------------------------------------
struct Shape {
  int tz, by, ry;
};

// With ev0/ev1 the dispatch itself carries the device's start and stop
// timestamps of the pass kernel (hipExtLaunchKernel), nothing else changes.
// fin: where the finish kernel after the pass stores the state (nullptr: no
// finish kernel; the next pass of the chain carries it).
template <typename T, int NF, bool FULL, int TZ, int BY, int RY>
hipError_t launch_shape(const ScalarArgs<T>& A, int nblocks, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                        DevState* fin) {
  if (ev0)
    hipExtLaunchKernelGGL((scalar_pass_kernel<T, NF, FULL, TZ, BY, RY>), dim3(nblocks), dim3(TZ * BY), 0, s, ev0,
                          ev1, 0, A);
  else
    hipLaunchKernelGGL((scalar_pass_kernel<T, NF, FULL, TZ, BY, RY>), dim3(nblocks), dim3(TZ * BY), 0, s, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fin) return e;
  hipLaunchKernelGGL((scalar_finish_kernel<T, NF, FULL>), dim3(1), dim3(kFinishThreads), 0, s, A, nblocks, fin);
  return hipGetLastError();
}

// Full-row tiles (stepping passes): tz = N, ry = 1, by y-rows per block.
template <typename T, int W, int NF, int NL, int BY>
hipError_t launch_rows(const ScalarArgs<T>& A, int nblocks, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                       DevState* fin) {
  if (ev0)
    hipExtLaunchKernelGGL((scalar_rows_kernel<T, W, NF, NL, BY>), dim3(nblocks), dim3(NL * BY), 0, s, ev0, ev1, 0, A);
  else
    hipLaunchKernelGGL((scalar_rows_kernel<T, W, NF, NL, BY>), dim3(nblocks), dim3(NL * BY), 0, s, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fin) return e;
  hipLaunchKernelGGL((scalar_finish_kernel<T, NF, false>), dim3(1), dim3(kFinishThreads), 0, s, A, nblocks, fin);
  return hipGetLastError();
}

// Stepping passes: every compiled tile shape (FP32 two-field is the
// production case; the other storage/field combinations get a subset).
// (the four- and eight-row shapes exceed 128 VGPRs with the coefficient pairs
// and spill the prefetched plane; they are not built for this case)
#define CL_SHAPES_MAIN(X, T, NF) \
  X(T, NF, 64, 4, 2)             \
  X(T, NF, 64, 8, 2)             \
  X(T, NF, 32, 8, 2)             \
  X(T, NF, 128, 8, 2)            \
  X(T, NF, 256, 4, 2)            \
  X(T, NF, 128, 4, 2)
#define CL_SHAPES_SMALL(X, T, NF) \
  X(T, NF, 64, 4, 2)              \
  X(T, NF, 32, 8, 2)              \
  X(T, NF, 32, 4, 4)

// full-row shapes (tz = N sites, by rows, ry = 1), 512 lanes, for N = 128,
// 256 and 512 (1024-lane blocks of these spill): four sites per lane in
// FP32 storage, two in FP64 (two FP32 sites per lane fit two blocks per CU
// but are slower: 113.9 against 109.7 us per pass at 256^3)
#define CL_ROWS_MAIN(X, NF) \
  X(float, NF, 128, 16, 4)  \
  X(float, NF, 256, 8, 4)   \
  X(float, NF, 512, 4, 4)
#define CL_ROWS_F64(X, NF)  \
  X(double, NF, 128, 8, 2)  \
  X(double, NF, 256, 4, 2)  \
  X(double, NF, 512, 2, 2)

static const Shape kShapesMain[] = {{64, 4, 2}, {64, 8, 2},  {32, 8, 2},  {128, 8, 2}, {256, 4, 2},
                                    {128, 4, 2}, {128, 16, 1}, {256, 8, 1}, {512, 4, 1}};
static const Shape kShapesSmall[] = {{64, 4, 2}, {32, 8, 2}, {32, 4, 4}};
static const Shape kShapesF64[] = {{64, 4, 2}, {32, 8, 2}, {32, 4, 4}, {128, 8, 1}, {256, 4, 1}, {512, 2, 1}};

// Observation passes always use the 32 x 16 tile with 8 planes, which
// divides every supported N.
static const int kObsTz = 32, kObsBy = 8, kObsRy = 2, kObsXc = 8;

int64_t scalar_obs_blocks(int N) {
  return (int64_t)(N / kObsTz) * (N / (kObsBy * kObsRy)) * (N / kObsXc);
}

template <typename T, int NF>
hipError_t launch_scalar_pass_t(const ScalarArgs<T>& A, const Shape& sh, int nblocks, hipStream_t s, bool full,
                                hipEvent_t ev0, hipEvent_t ev1, DevState* fin) {
  if (full) return launch_shape<T, NF, true, 32, 8, 2>(A, nblocks, s, ev0, ev1, fin);
#define X(TT, NFF, a, b, c) \
  if (sh.tz == a && sh.by == b && sh.ry == c)  \
    return launch_shape<TT, NFF, false, a, b, c>(A, nblocks, s, ev0, ev1, fin);
  if constexpr (std::is_same<T, float>::value && NF == 2) {
    CL_SHAPES_MAIN(X, T, NF)
#define XR(TT, NFF, n, b, w) \
  if (sh.tz == n && sh.by == b && sh.ry == 1) return launch_rows<TT, w, NFF, n / w, b>(A, nblocks, s, ev0, ev1, fin);
    CL_ROWS_MAIN(XR, NF)
  } else {
    CL_SHAPES_SMALL(X, T, NF)
    if constexpr (std::is_same<T, double>::value && NF == 2) {
      CL_ROWS_F64(XR, NF)
    }
#undef XR
  }
#undef X
  return hipErrorInvalidValue;
}

int num_shapes(int fp32, int nf) {
  if (nf == 2) return fp32 ? (int)(sizeof(kShapesMain) / sizeof(Shape)) : (int)(sizeof(kShapesF64) / sizeof(Shape));
  return (int)(sizeof(kShapesSmall) / sizeof(Shape));
}
void get_shape(int fp32, int nf, int i, int* tz, int* by, int* ry) {
  const Shape& sh = nf == 2 ? (fp32 ? kShapesMain[i] : kShapesF64[i]) : kShapesSmall[i];
  *tz = sh.tz;
  *by = sh.by;
  *ry = sh.ry;
}


// Launch one pass.  buffers: src/dst arrays [4] in storage precision.
hipError_t launch_scalar_pass(int fp32, int nf, const void* const* src, void* const* dst, int N, int tz,
                              int by, int ry, int xc, int swizzle, const double* phys, int expand,
                              const PassDesc& pd, double* partials, DevState* st, hipStream_t s,
                              int* nblocks_out, int full, hipEvent_t ev0, hipEvent_t ev1, const PrevPass& prev,
                              DevState* fin) {
  if (full && (prev.partials || !fin)) return hipErrorInvalidValue;  // observation passes finish themselves
  if ((pd.write != 0) == (full != 0)) return hipErrorInvalidValue;    // stepping passes store, observations do not
  if (full) {
    tz = kObsTz;
    by = kObsBy;
    ry = kObsRy;
    xc = kObsXc;
  }
  const Shape sh{tz, by, ry};
  const int ty = by * ry;
  const int nblocks = (N / tz) * (N / ty) * (N / xc);
  if (nblocks_out) *nblocks_out = nblocks;
  const int swz = (swizzle && (nblocks % 8 == 0)) ? 1 : 0;
  auto fill = [&](auto& A, auto* tag) {
    using TT = std::remove_pointer_t<decltype(tag)>;
    for (int i = 0; i < 4; ++i) {
      A.src[i] = static_cast<const TT*>(src[i]);
      A.dst[i] = static_cast<TT*>(dst[i]);
    }
    A.N = N;
    A.XC = xc;
    A.swizzle = swz;
    A.dx = phys[0];
    A.alpha = phys[1];
    A.fmp2 = phys[2];
    A.m2_0 = phys[3];
    A.m2_1 = phys[4];
    A.lam = phys[5];
    A.q = phys[6];
    A.h = phys[7];
    A.expand = expand;
    A.pd = pd;
    A.partials = partials;
    A.st = st;
    A.prev = prev;
  };
  if (fp32) {
    ScalarArgs<float> A;
    fill(A, (float*)nullptr);
    return nf == 1 ? launch_scalar_pass_t<float, 1>(A, sh, nblocks, s, full, ev0, ev1, fin)
                   : launch_scalar_pass_t<float, 2>(A, sh, nblocks, s, full, ev0, ev1, fin);
  } else {
    ScalarArgs<double> A;
    fill(A, (double*)nullptr);
    return nf == 1 ? launch_scalar_pass_t<double, 1>(A, sh, nblocks, s, full, ev0, ev1, fin)
                   : launch_scalar_pass_t<double, 2>(A, sh, nblocks, s, full, ev0, ev1, fin);
  }
}

// Finish kernel alone: the pass `pd` that wrote `nblocks` partial records
// started from state `in`; the result goes to `out` (the trailing finish of a
// chain of passes).
hipError_t launch_scalar_finish(int fp32, int nf, int N, const double* phys, int expand, const PassDesc& pd,
                                double* partials, int nblocks, DevState* in, DevState* out, hipStream_t s) {
  auto go = [&](auto* tag) -> hipError_t {
    using TT = std::remove_pointer_t<decltype(tag)>;
    ScalarArgs<TT> A = {};
    A.N = N;
    A.dx = phys[0];
    A.alpha = phys[1];
    A.fmp2 = phys[2];
    A.m2_0 = phys[3];
    A.m2_1 = phys[4];
    A.lam = phys[5];
    A.q = phys[6];
    A.h = phys[7];
    A.expand = expand;
    A.pd = pd;
    A.partials = partials;
    A.st = in;
    if (nf == 1)
      hipLaunchKernelGGL((scalar_finish_kernel<TT, 1, false>), dim3(1), dim3(kFinishThreads), 0, s, A, nblocks, out);
    else
      hipLaunchKernelGGL((scalar_finish_kernel<TT, 2, false>), dim3(1), dim3(kFinishThreads), 0, s, A, nblocks, out);
    return hipGetLastError();
  };
  return fp32 ? go((float*)nullptr) : go((double*)nullptr);
}

}  // namespace cl
