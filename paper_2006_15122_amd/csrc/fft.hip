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

template <typename R>
struct Cx {
  R x, y;
};

struct FFTPlan {
  int N;
  int nfac;
  int fac[16];
};

static FFTPlan make_plan(int N) {
  FFTPlan P;
  P.N = N;
  P.nfac = 0;
  int n = N;
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

// One batch of B lines along `axis`, transformed with exponent sign `sgn`
// (+1: forward of Sec. 3.1, -1: inverse without the 1/N^3), then scaled.
template <typename R>
__global__ __launch_bounds__(256) void fft_lines_kernel(Cx<R>* data, FFTPlan P, int axis, int B, double sgn,
                                                         double scale) {
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
  const double twopi = 6.283185307179586476925286766559;
  for (int f = 0; f < P.nfac; ++f) {
    const int Rr = P.fac[f];
    const int M = N / Rr;
    for (int t = tid; t < B * M; t += NT) {
      const int b = t / M, j = t % M, k = j % Ns;
      Cx<R> v[kMaxRadix];
      const double ang = sgn * twopi * (double)k / (double)(Ns * Rr);
      for (int r = 0; r < Rr; ++r) {
        Cx<R> x = in[b * N + j + r * M];
        if (r > 0 && k > 0) {
          double sv, cv;
          sincos(ang * r, &sv, &cv);
          x = cmul(x, Cx<R>{(R)cv, (R)sv});
        }
        v[r] = x;
      }
      Cx<R> o[kMaxRadix];
      if (Rr == 2) {
        o[0] = Cx<R>{v[0].x + v[1].x, v[0].y + v[1].y};
        o[1] = Cx<R>{v[0].x - v[1].x, v[0].y - v[1].y};
      } else if (Rr == 4) {
        // e^{sgn 2 pi i m r/4}: multiplication by sgn*i for m r = 1 (mod 4)
        const R s = (R)sgn;
        const Cx<R> a0{v[0].x + v[2].x, v[0].y + v[2].y}, a1{v[0].x - v[2].x, v[0].y - v[2].y};
        const Cx<R> b0{v[1].x + v[3].x, v[1].y + v[3].y}, b1{v[1].x - v[3].x, v[1].y - v[3].y};
        // i*s*b1 = (-s b1.y, s b1.x)
        o[0] = Cx<R>{a0.x + b0.x, a0.y + b0.y};
        o[2] = Cx<R>{a0.x - b0.x, a0.y - b0.y};
        o[1] = Cx<R>{a1.x - s * b1.y, a1.y + s * b1.x};
        o[3] = Cx<R>{a1.x + s * b1.y, a1.y - s * b1.x};
      } else {
        for (int m = 0; m < Rr; ++m) {
          double sx = 0.0, sy = 0.0;
          for (int r = 0; r < Rr; ++r) {
            double sv, cv;
            sincos(sgn * twopi * (double)((r * m) % Rr) / (double)Rr, &sv, &cv);
            sx += (double)v[r].x * cv - (double)v[r].y * sv;
            sy += (double)v[r].x * sv + (double)v[r].y * cv;
          }
          o[m] = Cx<R>{(R)sx, (R)sy};
        }
      }
      const int idxD = (j / Ns) * Ns * Rr + k;
      for (int r = 0; r < Rr; ++r) out[b * N + idxD + r * Ns] = o[r];
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

template <typename R>
static int fft3d(Cx<R>* data, int N, double sgn, double scale, hipStream_t s) {
  const FFTPlan P = make_plan(N);
  for (int f = 0; f < P.nfac; ++f)
    if (P.fac[f] > kMaxRadix) { set_error("FFT radix above 32"); return LAT_EINVAL; }
  int B = 32;
  while (B > 1 && (size_t)2 * B * N * sizeof(Cx<R>) > 65536) B >>= 1;
  const size_t shm = (size_t)2 * B * N * sizeof(Cx<R>);
  const int nblk = (int)((size_t)N * N / B);
  for (int axis = 2; axis >= 0; --axis) {
    const double sc = axis == 0 ? scale : 1.0;
    hipLaunchKernelGGL(fft_lines_kernel<R>, dim3(nblk), dim3(256), shm, s, data, P, axis, B, sgn, sc);
    CL_HIP(hipGetLastError());
  }
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

__device__ __forceinline__ int wrapk(int i, int N) { return i <= N / 2 ? i : i - N; }

// Per-block shell histograms of |f(n~)|^2, sum of |n~| and mode counts.
template <typename R>
__global__ __launch_bounds__(256) void bin_kernel(const Cx<R>* F, int N, int nbins, int64_t per_block,
                                                  double* pS, double* pK, unsigned long long* pC) {
  extern __shared__ unsigned char smem_raw[];
  double* hS = reinterpret_cast<double*>(smem_raw);
  double* hK = hS + nbins;
  unsigned long long* hC = reinterpret_cast<unsigned long long*>(hK + nbins);
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) { hS[b] = 0.0; hK[b] = 0.0; hC[b] = 0ull; }
  __syncthreads();
  const int64_t V = (int64_t)N * N * N;
  const int64_t i0 = (int64_t)blockIdx.x * per_block;
  const int64_t i1 = min(V, i0 + per_block);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const int i3 = (int)(i % N), i2 = (int)((i / N) % N), i1x = (int)(i / ((int64_t)N * N));
    const int n1 = wrapk(i1x, N), n2 = wrapk(i2, N), n3 = wrapk(i3, N);
    const int64_t n2s = (int64_t)n1 * n1 + (int64_t)n2 * n2 + (int64_t)n3 * n3;
    int b = (int)sqrt((double)n2s);
    while ((int64_t)(b + 1) * (b + 1) <= n2s) ++b;
    while ((int64_t)b * b > n2s) --b;
    const Cx<R> v = F[i];
    const double p = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    atomicAdd(&hS[b], p);
    atomicAdd(&hK[b], sqrt((double)n2s));
    atomicAdd(&hC[b], 1ull);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    pS[(size_t)blockIdx.x * nbins + b] = hS[b];
    pK[(size_t)blockIdx.x * nbins + b] = hK[b];
    pC[(size_t)blockIdx.x * nbins + b] = hC[b];
  }
}

// Sum the per-block histograms in block order and normalise (Sec. 3.1):
//   k[b] = k_IR <|n~|>_shell,
//   delta[b] = (k_IR b)^3/(2 pi^2) (dx/N)^3 S_b / (4 pi b^2)   (b >= 1).
__global__ void bin_sum_kernel(const double* pS, const double* pK, const unsigned long long* pC, int nblk,
                               int nbins, double kIR, double norm, double* S, double* K, double* D,
                               unsigned long long* C) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double s = 0.0, k = 0.0;
  unsigned long long c = 0;
  for (int j = 0; j < nblk; ++j) {
    s += pS[(size_t)j * nbins + b];
    k += pK[(size_t)j * nbins + b];
    c += pC[(size_t)j * nbins + b];
  }
  const double pi = 3.14159265358979323846264338327950288;
  S[b] = s;
  K[b] = c ? kIR * k / (double)c : 0.0;
  const double kb = kIR * (double)b;
  D[b] = b > 0 ? kb * kb * kb * norm * s / (4.0 * pi * (double)b * (double)b) : 0.0;
  C[b] = c;
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
  if (p.model == LAT_MODEL_U1) {
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
  if (p.model == LAT_MODEL_U1) {
    // V = lambda (phi0^2 + phi1^2)^2 / 4 + m2 (phi0^2 + phi1^2) / 2
    const double s = a * a + c * c, x = f == 0 ? a : c;
    return p.lambda * (s + 2.0 * x * x) + p.m2[0];
  }
  if (f == 0) return p.m2[0] + 3.0 * p.lambda * a * a + p.q * c * c;
  return p.m2[1] + p.q * a * a;
}

int run_fft3d(lattice* h, int sign, double scale) {
  return fft3d(reinterpret_cast<Cx<double>*>(h->fft), h->p.N, (double)sign, scale, h->stream);
}

// Homogeneous values plus (optionally) vacuum fluctuations for the scalar
// model, then b from the Hubble constraint with the full-lattice energies.
int init_state(lattice* h) {
  const lattice_params& p = h->p;
  if (p.model == LAT_MODEL_U1) return u1_init_state(h);
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
    rc = (p.model == LAT_MODEL_U1) ? u1_energies(h) : scalar_energies(h);
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

int spectrum_bins(lattice_t* h, int which, Bins* out) {
  const int N = h->p.N;
  const int nb = (int)std::floor(std::sqrt(3.0) * N / 2.0) + 1;
  int comp = -1;
  if (h->p.model == LAT_MODEL_SCALAR) {
    if (which >= 0 && which < h->p.nf) comp = which;
    else if (which >= 16 && which < 16 + h->p.nf) comp = h->p.nf + which - 16;
  } else {
    if (which >= 0 && which < 2) comp = which;                 // Re, Im of phi
    else if (which >= 16 && which < 18) comp = 2 + which - 16;  // Re, Im of pi
  }
  if (comp < 0) { set_error("spectrum: unknown field selector"); return LAT_EINVAL; }
  const int64_t V = (int64_t)N * N * N;
  const int threads = 256;
  const int blocks = (int)((V + threads - 1) / threads);
  Cx<double>* F = reinterpret_cast<Cx<double>*>(h->fft);
  const void* src = h->buf[h->cur][comp];
  if (h->p.precision == LAT_FP32)
    hipLaunchKernelGGL((real_to_complex_kernel<float, double>), dim3(blocks), dim3(threads), 0, h->stream,
                       (const float*)src, F, V);
  else
    hipLaunchKernelGGL((real_to_complex_kernel<double, double>), dim3(blocks), dim3(threads), 0, h->stream,
                       (const double*)src, F, V);
  CL_HIP(hipGetLastError());
  int rc = run_fft3d(h, +1, 1.0);
  if (rc) return rc;
  const int nblk = kSpecBlocks;
  const int64_t per = (V + nblk - 1) / nblk;
  double* pS = (double*)h->spec;
  double* pK = pS + (size_t)nblk * nb;
  unsigned long long* pC = (unsigned long long*)(pK + (size_t)nblk * nb);
  double* S = (double*)(pC + (size_t)nblk * nb);
  double* K = S + nb;
  double* D = K + nb;
  unsigned long long* C = (unsigned long long*)(D + nb);
  const size_t shm = (size_t)nb * 24;
  hipLaunchKernelGGL(bin_kernel<double>, dim3(nblk), dim3(256), shm, h->stream, F, N, nb, per, pS, pK, pC);
  CL_HIP(hipGetLastError());
  const double norm = std::pow(h->dx / N, 3.0) / (2.0 * M_PI * M_PI);
  hipLaunchKernelGGL(bin_sum_kernel, dim3((nb + 127) / 128), dim3(128), 0, h->stream, pS, pK, pC, nblk, nb,
                     h->p.kIR, norm, S, K, D, C);
  CL_HIP(hipGetLastError());
  *out = Bins{S, K, D, C, nb};
  return LAT_OK;
}

// log10 of the mode-averaged spectrum kbar^3 norm S_b / C_b at nk log-spaced
// k from kIR to kIR (nb - 1), linear in log k between the centres of shells
// b >= 1 with modes and positive power, constant beyond the end shells.
// One thread per output wavenumber; the shells are scanned in order.
__global__ void logk_kernel(const double* S, const double* K, const unsigned long long* C, int nb, double norm,
                            double kIR, int nk, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nk) return;
  const double kmax = kIR * (double)(nb - 1);
  const double x = log10(kIR) + (log10(kmax) - log10(kIR)) * (double)j / (double)(nk - 1);
  double x0 = 0.0, y0 = 0.0, last = 0.0;
  bool have = false, done = false;
  double res = 0.0;
  for (int b = 1; b < nb && !done; ++b) {
    if (C[b] == 0ull || !(S[b] > 0.0)) continue;
    const double kb = K[b];
    const double xb = log10(kb);
    const double yb = log10(kb * kb * kb * norm * S[b] / (double)C[b]);
    if (!have) {
      if (x <= xb) { res = yb; done = true; }
    } else if (x <= xb) {
      res = y0 + (x - x0) / (xb - x0) * (yb - y0);
      done = true;
    }
    have = true;
    x0 = xb;
    y0 = yb;
    last = yb;
  }
  if (!done) res = have ? last : -INFINITY;
  out[j] = (float)res;
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
  hipLaunchKernelGGL(logk_kernel, dim3((nk + 63) / 64), dim3(64), 0, h->stream, B.S, B.K, B.C, B.nb, norm,
                     h->p.kIR, nk, dev_out);
  CL_HIP(hipGetLastError());
  return LAT_OK;
}
