/*
 * Plain FP64 CPU oracle for the lattice method of Figueroa, Florio,
 * Torrenti, Valkenburg, "The art of simulating the early Universe - Part I"
 * (arXiv:2006.15122).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * cpu_baseline leg of the benchmark load this library.  The HIP product path
 * shares no code with it and never links it.
 *
 * Every loop below is one line of the paper's schemes, written out plainly:
 * a kick pass, a reduction pass, a drift pass, in the order the paper gives.
 * No fusion, no blocking.  Reductions use one partial sum per x-plane, added
 * in plane order, so results do not depend on the thread count.
 *
 * Lattice layout: site (x,y,z), 0 <= x,y,z < N, linear index (x*N+y)*N+z;
 * periodic boundaries (Sec. 3.1).  Fields are stored field-major:
 * phi[f*N^3 + site].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,   */
/* SC'11, "Parallel random numbers: as easy as 1, 2, 3").  Used only to  */
/* draw the Rayleigh moduli and uniform phases of the initial            */
/* fluctuations (Sec. 7.1).                                              */
/* ------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
    philox_round(c, k);
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Fill out[4*i .. 4*i+3] with Philox(counter = (i_lo, i_hi, c2, c3),
   key = (seed_lo, seed_hi)) for i = 0..n-1. */
void orc_philox_stream(uint64_t seed, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), c2, c3};
    orc_philox4x32_10(ctr, key, out + 4 * i);
  }
}

/* ------------------------------------------------------------------ */
/* Real scalar fields in an FLRW background (Sec. 4).                   */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t N;        /* sites per side */
  int32_t nf;       /* number of real fields: 1 (phi) or 2 (phi, chi) */
  int32_t expand;   /* 1: self-consistent a(eta); 0: flat, a = 1, b = 0 */
  int32_t pad;
  double dx;        /* lattice spacing in program units, 2 pi / (kIR N) */
  double alpha;     /* alpha-time exponent, d eta = a^-alpha w* dt */
  double fmp2;      /* (f_star/m_p)^2 */
  double m2[2];     /* program masses: V contains m2[i] phi_i^2 / 2 */
  double lambda;    /* V contains lambda phi^4 / 4 */
  double q;         /* V contains q phi^2 chi^2 / 2 */
} orc_scalar;

static inline int64_t site(int N, int x, int y, int z) {
  x = (x + N) % N; y = (y + N) % N; z = (z + N) % N;
  return ((int64_t)x * N + y) * N + z;
}

/* Program potential and its terms (Sec. 4.5.1: E_V and E_{V_a}). */
static double pot_terms(const orc_scalar* m, double phi, double chi, double t[3]) {
  t[0] = 0.5 * m->m2[0] * phi * phi + (m->nf > 1 ? 0.5 * m->m2[1] * chi * chi : 0.0);
  t[1] = 0.25 * m->lambda * phi * phi * phi * phi;
  t[2] = m->nf > 1 ? 0.5 * m->q * phi * phi * chi * chi : 0.0;
  return t[0] + t[1] + t[2];
}

/* dV/dphi_f */
static double dpot(const orc_scalar* m, int f, double phi, double chi) {
  if (f == 0) {
    double d = m->m2[0] * phi + m->lambda * phi * phi * phi;
    if (m->nf > 1) d += m->q * chi * chi * phi;
    return d;
  }
  return m->m2[1] * chi + m->q * phi * phi * chi;
}

/* Field kernel of the scalar Verlet schemes (Sec. 4.3, Hamiltonian form):
   K_f = a^{1+alpha} sum_k Delta^-_k Delta^+_k phi_f - a^{3+alpha} V_{,phi_f}. */
void orc_scalar_kernel(const orc_scalar* m, double a, const double* phi, double* K) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  const double cl = pow(a, 1.0 + m->alpha) / (m->dx * m->dx);
  const double cp = pow(a, 3.0 + m->alpha);
  for (int f = 0; f < m->nf; ++f) {
    const double* p = phi + f * V;
#pragma omp parallel for schedule(static)
    for (int x = 0; x < N; ++x)
      for (int y = 0; y < N; ++y)
        for (int z = 0; z < N; ++z) {
          const int64_t s = site(N, x, y, z);
          const double lap = p[site(N, x + 1, y, z)] + p[site(N, x - 1, y, z)]
                           + p[site(N, x, y + 1, z)] + p[site(N, x, y - 1, z)]
                           + p[site(N, x, y, z + 1)] + p[site(N, x, y, z - 1)]
                           - 6.0 * p[s];
          const double chi = m->nf > 1 ? phi[V + s] : 0.0;
          K[f * V + s] = cl * lap - cp * dpot(m, f, phi[s], chi);
        }
  }
}

/* Raw volume averages needed by the energies (Sec. 4.5), per field f:
   out[4f+0] = <pi_f^2>, out[4f+1] = <sum_k (phi_f(n+k) - phi_f(n))^2> (no 1/dx^2),
   out[4f+2] = <phi_f>,  out[4f+3] = <phi_f^2>;
   then out[4nf+0..2] = <V_mass>, <V_quartic>, <V_int>.
   pi may be NULL (then <pi^2> = 0). */
void orc_scalar_sums(const orc_scalar* m, const double* phi, const double* pi, double* out) {
  const int N = m->N, nf = m->nf;
  const int64_t V = (int64_t)N * N * N;
  const int nacc = 4 * nf + 3;
  double* part = (double*)calloc((size_t)N * nacc, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int x = 0; x < N; ++x) {
    double* acc = part + (size_t)x * nacc;
    for (int y = 0; y < N; ++y)
      for (int z = 0; z < N; ++z) {
        const int64_t s = site(N, x, y, z);
        for (int f = 0; f < nf; ++f) {
          const double* p = phi + f * V;
          const double gx = p[site(N, x + 1, y, z)] - p[s];
          const double gy = p[site(N, x, y + 1, z)] - p[s];
          const double gz = p[site(N, x, y, z + 1)] - p[s];
          if (pi) acc[4 * f + 0] += pi[f * V + s] * pi[f * V + s];
          acc[4 * f + 1] += gx * gx + gy * gy + gz * gz;
          acc[4 * f + 2] += p[s];
          acc[4 * f + 3] += p[s] * p[s];
        }
        double t[3];
        pot_terms(m, phi[s], nf > 1 ? phi[V + s] : 0.0, t);
        acc[4 * nf + 0] += t[0];
        acc[4 * nf + 1] += t[1];
        acc[4 * nf + 2] += t[2];
      }
  }
  for (int k = 0; k < nacc; ++k) {
    double s = 0.0;
    for (int x = 0; x < N; ++x) s += part[(size_t)x * nacc + k];
    out[k] = s / (double)V;
  }
  free(part);
}

/* Energies in program units (Sec. 4.3, E_K = sum <pi^2>/(2a^6),
   E_G = sum <(grad phi)^2>/(2a^2), E_V = <V>).
   e[0]=E_K, e[1]=E_G, e[2]=E_V, e[3..5]=V terms, then per field f:
   e[6+4f]=E_K^f, e[7+4f]=E_G^f, e[8+4f]=<phi_f>, e[9+4f]=<phi_f^2>. */
void orc_scalar_energies(const orc_scalar* m, double a, const double* sums, double* e) {
  const int nf = m->nf;
  const double a6 = pow(a, 6.0), a2 = a * a, dx2 = m->dx * m->dx;
  e[0] = e[1] = 0.0;
  for (int f = 0; f < nf; ++f) {
    const double ek = sums[4 * f + 0] / (2.0 * a6);
    const double eg = sums[4 * f + 1] / (2.0 * a2 * dx2);
    e[6 + 4 * f] = ek;
    e[7 + 4 * f] = eg;
    e[8 + 4 * f] = sums[4 * f + 2];
    e[9 + 4 * f] = sums[4 * f + 3];
    e[0] += ek;
    e[1] += eg;
  }
  e[3] = sums[4 * nf + 0];
  e[4] = sums[4 * nf + 1];
  e[5] = sums[4 * nf + 2];
  e[2] = e[3] + e[4] + e[5];
}

/* Scale-factor kernel (Sec. 4.3): b' = K_a = (1/3)(f_star/m_p)^2 a^{1+2alpha}
   [ (alpha-2) E_K + alpha E_G + (alpha+1) E_V ]. */
double orc_Ka(const orc_scalar* m, double a, double EK, double EG, double EV) {
  const double al = m->alpha;
  return m->fmp2 / 3.0 * pow(a, 1.0 + 2.0 * al) * ((al - 2.0) * EK + al * EG + (al + 1.0) * EV);
}

/* Hubble constraint right-hand side (Sec. 4.3):
   (1/3)(f_star/m_p)^2 a^{2(alpha+1)} (E_K + E_G + E_V). */
double orc_hc_rhs(const orc_scalar* m, double a, double rho) {
  return m->fmp2 / 3.0 * pow(a, 2.0 * (m->alpha + 1.0)) * rho;
}

static void energies_of(const orc_scalar* m, double a, const double* phi, const double* pi, double* e) {
  double s[4 * 2 + 3];
  orc_scalar_sums(m, phi, pi, s);
  orc_scalar_energies(m, a, s, e);
}

/* One velocity-Verlet sub-step of weight w (Sec. 4.4, VVn with expansion),
   in the paper's order:
     b_{1/2}  = b + (w h/2) K_a[a, E(phi, pi)]
     pi_{1/2} = pi + (w h/2) K[a, phi]
     a'       = a + w h b_{1/2},  a_{1/2} = (a + a')/2
     phi'     = phi + w h pi_{1/2} a_{1/2}^{-(3-alpha)}
     pi'      = pi_{1/2} + (w h/2) K[a', phi']
     b'       = b_{1/2} + (w h/2) K_a[a', E(phi', pi')]
   scratch must hold nf*N^3 doubles. */
void orc_vv_substep(const orc_scalar* m, double* phi, double* pi, double* a, double* b,
                    double wh, double* K) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  const int64_t n = m->nf * V;
  double e[6 + 8];
  if (m->expand) {
    energies_of(m, *a, phi, pi, e);
    *b = *b + 0.5 * wh * orc_Ka(m, *a, e[0], e[1], e[2]);
  }
  orc_scalar_kernel(m, *a, phi, K);
  for (int64_t i = 0; i < n; ++i) pi[i] = pi[i] + 0.5 * wh * K[i];
  double anew = *a, ahalf = *a;
  if (m->expand) {
    anew = *a + wh * (*b);
    ahalf = 0.5 * (*a + anew);
  }
  const double cdrift = wh * pow(ahalf, -(3.0 - m->alpha));
  for (int64_t i = 0; i < n; ++i) phi[i] = phi[i] + cdrift * pi[i];
  *a = anew;
  orc_scalar_kernel(m, *a, phi, K);
  for (int64_t i = 0; i < n; ++i) pi[i] = pi[i] + 0.5 * wh * K[i];
  if (m->expand) {
    energies_of(m, *a, phi, pi, e);
    *b = *b + 0.5 * wh * orc_Ka(m, *a, e[0], e[1], e[2]);
  }
}

/* nsteps full steps of VVn: each step is s sub-steps with weights w[0..s-1]
   (s = 1, w = {1}: VV2; s = 3: VV4, weights of the Yoshida table). */
void orc_vv_steps(const orc_scalar* m, double* phi, double* pi, double* a, double* b,
                  double h, const double* w, int s, int64_t nsteps) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* K = (double*)malloc(sizeof(double) * m->nf * V);
  for (int64_t it = 0; it < nsteps; ++it)
    for (int p = 0; p < s; ++p) orc_vv_substep(m, phi, pi, a, b, w[p] * h, K);
  free(K);
}

/* Staggered leapfrog, scheme III of Sec. 4.2.1 (pi = a^{3-alpha} phi').
   State: phi_n, a_n at integer time; pi_{n-1/2}, b_{n-1/2} at half-integer time.
   Start-up from a synchronised state (phi_0, pi_0, a_0, b_0):
     pi_{-1/2} = pi_0 - (h/2) K[a_0, phi_0]
     b_{-1/2}  = b_0  - (h/2) K_a[a_0, E(phi_0, pi_0)]                         */
void orc_lf_startup(const orc_scalar* m, double* phi, double* pi, double* a, double* b, double h) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  const int64_t n = m->nf * V;
  double* K = (double*)malloc(sizeof(double) * n);
  double e[6 + 8];
  if (m->expand) {
    energies_of(m, *a, phi, pi, e);
    *b = *b - 0.5 * h * orc_Ka(m, *a, e[0], e[1], e[2]);
  }
  orc_scalar_kernel(m, *a, phi, K);
  for (int64_t i = 0; i < n; ++i) pi[i] = pi[i] - 0.5 * h * K[i];
  free(K);
}

/* Averaged kinetic energy at integer time n from the two staggered momenta,
   both weighted with a_n^6 (the paper's average of E_K(n-1/2) and
   E_K(n+1/2), with the scale factor taken at n so that the update stays
   explicit). */
static double lf_avg_EK(const orc_scalar* m, double a, const double* pim, const double* pip) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double s = 0.0;
  for (int f = 0; f < m->nf; ++f) {
    double sm = 0.0, sp = 0.0;
    for (int64_t i = 0; i < V; ++i) { sm += pim[f * V + i] * pim[f * V + i]; sp += pip[f * V + i] * pip[f * V + i]; }
    s += (sm + sp) / (double)V;
  }
  return s / (4.0 * pow(a, 6.0));
}

/* One staggered-leapfrog step, scheme III:
     pi_{n+1/2} = pi_{n-1/2} + h K[a_n, phi_n]
     b_{n+1/2}  = b_{n-1/2} + h K_a[a_n, avgE_K(n), E_G(phi_n), E_V(phi_n)]
     a_{n+1}    = a_n + h b_{n+1/2}
     phi_{n+1}  = phi_n + h pi_{n+1/2} a_{n+1/2}^{-(3-alpha)}                */
void orc_lf_steps(const orc_scalar* m, double* phi, double* pi, double* a, double* b,
                  double h, int64_t nsteps) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  const int64_t n = m->nf * V;
  double* K = (double*)malloc(sizeof(double) * n);
  double* pold = (double*)malloc(sizeof(double) * n);
  double e[6 + 8];
  for (int64_t it = 0; it < nsteps; ++it) {
    orc_scalar_kernel(m, *a, phi, K);
    memcpy(pold, pi, sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) pi[i] = pi[i] + h * K[i];
    double anew = *a, ahalf = *a;
    if (m->expand) {
      energies_of(m, *a, phi, NULL, e);
      const double ekbar = lf_avg_EK(m, *a, pold, pi);
      *b = *b + h * orc_Ka(m, *a, ekbar, e[1], e[2]);
      anew = *a + h * (*b);
      ahalf = 0.5 * (*a + anew);
    }
    const double cdrift = h * pow(ahalf, -(3.0 - m->alpha));
    for (int64_t i = 0; i < n; ++i) phi[i] = phi[i] + cdrift * pi[i];
    *a = anew;
  }
  free(pold);
  free(K);
}

/* Observables of a staggered state (phi_n, pi_{n-1/2}, a_n, b_{n-1/2}) at the
   integer time n.  The momentum half a step ahead, pi_{n+1/2}, and b_{n+1/2}
   are formed as in the next step but not stored.  Output as
   orc_scalar_energies, followed by e[6+4nf] = b_n = (b_{n-1/2}+b_{n+1/2})/2
   and e[7+4nf] = Hubble-constraint residual at n. */
void orc_lf_observe(const orc_scalar* m, const double* phi, const double* pi, double a, double b,
                    double h, double* e) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  const int64_t n = m->nf * V;
  double* K = (double*)malloc(sizeof(double) * n);
  double* pip = (double*)malloc(sizeof(double) * n);
  orc_scalar_kernel(m, a, phi, K);
  for (int64_t i = 0; i < n; ++i) pip[i] = pi[i] + h * K[i];
  double s[4 * 2 + 3];
  orc_scalar_sums(m, phi, NULL, s);
  /* per-field averaged kinetic term */
  for (int f = 0; f < m->nf; ++f) {
    double sm = 0.0, sp = 0.0;
    for (int64_t i = 0; i < V; ++i) { sm += pi[f * V + i] * pi[f * V + i]; sp += pip[f * V + i] * pip[f * V + i]; }
    s[4 * f + 0] = 0.5 * (sm + sp) / (double)V;
  }
  orc_scalar_energies(m, a, s, e);
  const int nf = m->nf;
  double bn = b, hc = 0.0;
  if (m->expand) {
    const double bp = b + h * orc_Ka(m, a, e[0], e[1], e[2]);
    bn = 0.5 * (b + bp);
    const double rhs = orc_hc_rhs(m, a, e[0] + e[1] + e[2]);
    hc = fabs(bn * bn - rhs) / (bn * bn);
  }
  e[6 + 4 * nf] = bn;
  e[7 + 4 * nf] = hc;
  free(pip);
  free(K);
}

/* Observables of a synchronised state (Sec. 4.5), output as
   orc_scalar_energies followed by the Hubble-constraint residual
   |b^2 - rhs| / b^2 (Sec. 4.4, HC of the VVn scheme). */
void orc_sync_observe(const orc_scalar* m, const double* phi, const double* pi, double a, double b,
                      double* e) {
  energies_of(m, a, phi, pi, e);
  double hc = 0.0;
  if (m->expand) {
    const double rhs = orc_hc_rhs(m, a, e[0] + e[1] + e[2]);
    hc = fabs(b * b - rhs) / (b * b);
  }
  e[6 + 4 * m->nf] = b;
  e[7 + 4 * m->nf] = hc;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
