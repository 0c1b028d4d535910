// Shared declarations of the HIP lattice library (device and host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/cosmolat.h"

namespace cl {

// Thread-local error text, set by every failing entry point.
void set_error(const std::string& msg);

#define CL_HIP(call)                                                              \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess) {                                                       \
      ::cl::set_error(std::string(#call) + ": " + hipGetErrorString(_e));         \
      return LAT_EHIP;                                                            \
    }                                                                             \
  } while (0)

// Device-resident homogeneous state and observables of one lattice.
// Written only by the last-arriving block of a pass (one thread), read by all
// blocks of the next pass.
struct DevState {
  double a;          // scale factor at the current (sub-)step time
  double b;          // a' (half a step ahead inside a run of passes)
  double eta;        // program time of a
  double aux[5];     // reserved
  lattice_obs obs;   // observables of the last pass
  unsigned int counter;   // arrival counter of the pass in flight
  int nonfinite;          // set when a volume average is NaN/Inf
};

// Parameters of one fused pass (Sec. 3.3.2/4.3.2 velocity Verlet with merged
// kicks; Sec. 4.2.1 staggered leapfrog):
//   a'   = a + wd h b
//   phi  = phi + wd h pi a_mid^{-(3-alpha)},       a_mid = (a + a')/2
//   K    = a'^{1+alpha} lap(phi) - a'^{3+alpha} V_{,phi}
//   pi   = pi + (wk1 + wk2) h K
//   b    = b + (wk1 + wk2) h K_a(a', E)
// In VV mode E_K is taken from pi + wk1 h K (the synchronised momentum); in
// LF mode from the mean of <pi_in^2> and <pi_out^2>.
enum PassMode { MODE_VV = 0, MODE_LF = 1 };

// A per-pass coefficient (h a^p, a^p / dx^2, ...) carried as the unevaluated
// sum hi + lo of two storage-precision numbers, which equals its FP64 value to
// about 2^-48 relative.  Rounding the coefficient itself to FP32 would change
// every site the same way every pass (a relative error of up to 6e-8 in the
// time step or a coupling), a coherent perturbation that the resonant growth
// amplifies like a change of the physics; the rounding of the products is
// random from site to site and averages out of the volume observables.
template <typename T>
struct Coef {
  T hi, lo;
};
template <typename T>
__host__ __device__ inline Coef<T> coef(double v) {
  const T hi = (T)v;
  return Coef<T>{hi, (T)(v - (double)hi)};
}
// The same pair moved to scalar registers: every lane of a wave computes the
// same coefficient (from a and b, which a chained pass reads out of LDS), so
// the first lane's value is every lane's.
__device__ __forceinline__ float wave_uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double wave_uniform(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// a^p for the scale-factor powers of the passes and their finishes, p = k +
// m alpha: an integer whenever alpha is (conformal time, alpha = 1, say),
// and an integer power of magnitude up to 8 is formed by repeated squaring (a
// few ulp from pow, at a fraction of its dependent FP64 chain, which sits on
// the critical path of every chained pass); other exponents take pow.
__device__ __forceinline__ double apow(double a, double p) {
  if (p == rint(p) && fabs(p) <= 8.0) {
    double r = 1.0, x = a;
    for (int k = (int)fabs(p); k; k >>= 1) {
      if (k & 1) r *= x;
      x *= x;
    }
    return p < 0.0 ? 1.0 / r : r;
  }
  return pow(a, p);
}
template <typename T>
__device__ __forceinline__ Coef<T> ucoef(double v) {
  const Coef<T> c = coef<T>(v);
  return Coef<T>{wave_uniform(c.hi), wave_uniform(c.lo)};
}
// acc + c x.  The increment c x is formed first (hi x + lo x, one rounding)
// and then added: adding lo x after hi x had been added to acc would round
// back to the same number, since lo x is below half an ulp of the sum, and
// leave the coefficient's rounding in place.
template <typename T>
__device__ __forceinline__ T fma_c(const Coef<T>& c, T x, T acc) {
  if constexpr (sizeof(T) == sizeof(double)) return fma(c.hi, x, acc);
  return acc + fmaf(c.hi, x, c.lo * x);
}
// c x
template <typename T>
__device__ __forceinline__ T mul_c(const Coef<T>& c, T x) {
  if constexpr (sizeof(T) == sizeof(double)) return c.hi * x;
  return fmaf(c.hi, x, c.lo * x);
}

struct PassDesc {
  double wd, wk1, wk2;
  int mode;
  int write;    // store phi and pi into the destination buffer
  int update;   // store a, b, eta into DevState
};

// The finish of the previous pass, carried by the next pass of a chain: every
// block reduces that pass's partial records itself (same fixed order, so the
// same a and b in every block) and block 0 stores the resulting state in
// `out`.  partials == nullptr: nothing pending, a and b come from st.
struct PrevPass {
  const double* partials;
  int nblocks;
  PassDesc pd;
  DevState* out;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), device and host.
struct Philox4 {
  uint32_t v[4];
};

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = 0xD2511F53ull * (uint64_t)c0;
    const uint64_t p1 = 0xCD9E8D57ull * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Philox4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

}  // namespace cl
