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

/* Program potential and its terms (Sec. 4.4.1: E_V and E_{V_a}). */
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

/* Field kernel of the scalar Verlet schemes (Sec. 4.2.3, Hamiltonian form):
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

/* Raw volume averages needed by the energies (Sec. 4.4), per field f:
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

/* Energies in program units (Sec. 4.4.1, E_K = sum <pi^2>/(2a^6),
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

/* Scale-factor kernel (Sec. 4.3.2): b' = K_a = (1/3)(f_star/m_p)^2 a^{1+2alpha}
   [ (alpha-2) E_K + alpha E_G + (alpha+1) E_V ]. */
double orc_Ka(const orc_scalar* m, double a, double EK, double EG, double EV) {
  const double al = m->alpha;
  return m->fmp2 / 3.0 * pow(a, 1.0 + 2.0 * al) * ((al - 2.0) * EK + al * EG + (al + 1.0) * EV);
}

/* Hubble constraint right-hand side (Sec. 4.3.2):
   (1/3)(f_star/m_p)^2 a^{2(alpha+1)} (E_K + E_G + E_V). */
double orc_hc_rhs(const orc_scalar* m, double a, double rho) {
  return m->fmp2 / 3.0 * pow(a, 2.0 * (m->alpha + 1.0)) * rho;
}

static void energies_of(const orc_scalar* m, double a, const double* phi, const double* pi, double* e) {
  double s[4 * 2 + 3];
  orc_scalar_sums(m, phi, pi, s);
  orc_scalar_energies(m, a, s, e);
}

/* One velocity-Verlet sub-step of weight w (Sec. 4.3.2, VVn with expansion),
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

/* Observables of a synchronised state (Sec. 4.4), output as
   orc_scalar_energies followed by the Hubble-constraint residual
   |b^2 - rhs| / b^2 (Sec. 4.3.2, HC of the VVn scheme). */
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

/* ------------------------------------------------------------------ */
/* Complex scalar with compact U(1) links (Sec. 5.1, 5.3; toolkit of   */
/* Sec. 3.2.2).  phi = (phi_0 + i phi_1)/sqrt 2 is stored as (Re, Im);  */
/* link V_i(n) = exp(-i e dx A_i) lives on n + i/2, stored (Re, Im);    */
/* pi_A,i is one real per link.  Plaquette                              */
/*   V_ij(n) = V_i(n) V_j(n+i) conj V_i(n+j) conj V_j(n).               */
/* With noncompact = 1 (Sec. 5.2) the link array holds the real gauge  */
/* field A_i(n) instead (3 N^3), V_i = exp(-i e dx A_i) is formed where  */
/* the scalar needs it, and the gauge sector is the quadratic one:     */
/* magnetic kernel sum_j (D-_j D+_j A_i - D-_j D+_i A_j), energy        */
/* sum_{i<j} F_ij^2 / 2 with F_ij = D+_i A_j - D+_j A_i, drift          */
/* A += h piA / a_mid^{1-alpha}.                                       */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t N, expand, noncompact, pad1;
  double dx, alpha, fmp2;
  double lambda;   /* V = lambda |phi|^4 + m2 |phi|^2 */
  double m2;
  double e;        /* gauge coupling g_A Q_A */
  double wf2;      /* (w_star/f_star)^2 */
} orc_u1;

typedef struct { double re, im; } cpx;
static inline cpx cmk(double r, double i) { cpx c = {r, i}; return c; }
static inline cpx cmul_(cpx a, cpx b) { return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static inline cpx cconj_(cpx a) { return cmk(a.re, -a.im); }

/* array views: phi[c*V + s] (c = 0 Re, 1 Im); links[(2*i + c)*V + s] */
static inline cpx phi_at(const double* phi, int64_t V, int64_t s) { return cmk(phi[s], phi[V + s]); }
static inline cpx link_c(const double* L, int64_t V, int i, int64_t s) { return cmk(L[(2 * i) * V + s], L[(2 * i + 1) * V + s]); }

static int64_t shift(int N, int64_t s, int dir, int step) {
  int x = (int)(s / ((int64_t)N * N)), y = (int)((s / N) % N), z = (int)(s % N);
  if (dir == 0) x += step; else if (dir == 1) y += step; else z += step;
  return site(N, x, y, z);
}

/* the link V_i(n) of either formulation */
static cpx link_at(const orc_u1* m, const double* L, int64_t V, int i, int64_t s) {
  if (!m->noncompact) return link_c(L, V, i, s);
  const double t = -m->e * m->dx * L[i * V + s];
  return cmk(cos(t), sin(t));
}

static cpx plaquette(const orc_u1* m, const double* L, int i, int j, int64_t s) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  const cpx a = link_at(m, L, V, i, s);
  const cpx b = link_at(m, L, V, j, shift(N, s, i, 1));
  const cpx c = cconj_(link_at(m, L, V, i, shift(N, s, j, 1)));
  const cpx d = cconj_(link_at(m, L, V, j, s));
  return cmul_(cmul_(a, b), cmul_(c, d));
}

/* Non-compact field strength F_ij(n) = D+_i A_j(n) - D+_j A_i(n) (Sec. 5.2). */
static double nc_F(const orc_u1* m, const double* A, int i, int j, int64_t s) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  return ((A[j * V + shift(N, s, i, 1)] - A[j * V + s]) - (A[i * V + shift(N, s, j, 1)] - A[i * V + s])) / m->dx;
}

/* Non-compact magnetic kernel sum_j (D-_j D+_j A_i - D-_j D+_i A_j)(n) (Sec. 5.2),
   each term written out from the forward and backward differences. */
static double nc_magnetic(const orc_u1* m, const double* A, int i, int64_t s) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  const double dx2 = m->dx * m->dx;
  double r = 0.0;
  for (int j = 0; j < 3; ++j) {
    const int64_t sjp = shift(N, s, j, 1), sjm = shift(N, s, j, -1);
    /* D-_j D+_j A_i */
    const double djj = (A[i * V + sjp] - 2.0 * A[i * V + s] + A[i * V + sjm]) / dx2;
    /* D-_j D+_i A_j = [D+_i A_j](n) - [D+_i A_j](n - j), over dx */
    const double dpi_n = A[j * V + shift(N, s, i, 1)] - A[j * V + s];
    const double dpi_m = A[j * V + shift(N, sjm, i, 1)] - A[j * V + sjm];
    r += djj - (dpi_n - dpi_m) / dx2;
  }
  return r;
}

/* Kernels of the compact U(1) scheme (Sec. 5.1 kernels, Sec. 5.3 gauge kernel):
   K_phi   = -a^{3+alpha} (2 lambda |phi|^2 + m2) phi
             + a^{1+alpha} sum_i (V_i phi_{+i} - 2 phi + conj V_i(n-i) phi_{-i}) / dx^2
   K_{A,i} = a^{1+alpha} (2 e / dx) (f_star/w_star)^2 Im[conj phi V_i phi_{+i}]
             + a^{alpha-1} / (e dx^3) sum_{j != i} (Im V_ij(n) - Im V_ij(n-j))          */
void orc_u1_kernels(const orc_u1* m, double a, const double* phi, const double* L, double* Kphi, double* KA) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  const double cl = pow(a, 1.0 + m->alpha) / (m->dx * m->dx);
  const double cp = pow(a, 3.0 + m->alpha);
  const double cj = pow(a, 1.0 + m->alpha) * 2.0 * m->e / m->dx / m->wf2;
  const double cb = pow(a, m->alpha - 1.0) / (m->e * m->dx * m->dx * m->dx);
  const double cbn = pow(a, m->alpha - 1.0);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < N; ++x)
    for (int y = 0; y < N; ++y)
      for (int z = 0; z < N; ++z) {
        const int64_t s = site(N, x, y, z);
        const cpx p = phi_at(phi, V, s);
        cpx lap = cmk(-6.0 * p.re, -6.0 * p.im);
        for (int i = 0; i < 3; ++i) {
          const int64_t sp = shift(N, s, i, 1), sm = shift(N, s, i, -1);
          const cpx f = cmul_(link_at(m, L, V, i, s), phi_at(phi, V, sp));
          const cpx b = cmul_(cconj_(link_at(m, L, V, i, sm)), phi_at(phi, V, sm));
          lap.re += f.re + b.re;
          lap.im += f.im + b.im;
        }
        const double r2 = p.re * p.re + p.im * p.im;
        const double dv = 2.0 * m->lambda * r2 + m->m2;
        Kphi[s] = cl * lap.re - cp * dv * p.re;
        Kphi[V + s] = cl * lap.im - cp * dv * p.im;
        for (int i = 0; i < 3; ++i) {
          const cpx cur = cmul_(cconj_(p), cmul_(link_at(m, L, V, i, s), phi_at(phi, V, shift(N, s, i, 1))));
          if (m->noncompact) {
            KA[i * V + s] = cj * cur.im + cbn * nc_magnetic(m, L, i, s);
            continue;
          }
          double mag = 0.0;
          for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            mag += plaquette(m, L, i, j, s).im - plaquette(m, L, i, j, shift(N, s, j, -1)).im;
          }
          KA[i * V + s] = cj * cur.im + cb * mag;
        }
      }
}

/* Raw volume averages (Sec. 5.4): out[0] = <|pi|^2>, out[1] = <sum_i |V_i phi_{+i} - phi|^2>
   (no 1/dx^2), out[2] = <lambda |phi|^4>, out[3] = <m2 |phi|^2>, out[4] = <sum_i piA_i^2>,
   out[5] = <sum_{i<j} (1 - Re V_ij)> (non-compact: <sum_{i<j} F_ij^2>), out[6] = <Re phi>,
   out[7] = <Im phi>, out[8] = <|phi|^2>. */
void orc_u1_sums(const orc_u1* m, const double* phi, const double* pi, const double* L, const double* piA,
                 double* out) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  const int nacc = 9;
  double* part = (double*)calloc((size_t)N * nacc, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int x = 0; x < N; ++x) {
    double* acc = part + (size_t)x * nacc;
    for (int y = 0; y < N; ++y)
      for (int z = 0; z < N; ++z) {
        const int64_t s = site(N, x, y, z);
        const cpx p = phi_at(phi, V, s);
        if (pi) acc[0] += pi[s] * pi[s] + pi[V + s] * pi[V + s];
        for (int i = 0; i < 3; ++i) {
          const cpx f = cmul_(link_at(m, L, V, i, s), phi_at(phi, V, shift(N, s, i, 1)));
          acc[1] += (f.re - p.re) * (f.re - p.re) + (f.im - p.im) * (f.im - p.im);
          if (piA) acc[4] += piA[i * V + s] * piA[i * V + s];
        }
        const double r2 = p.re * p.re + p.im * p.im;
        acc[2] += m->lambda * r2 * r2;
        acc[3] += m->m2 * r2;
        for (int i = 0; i < 3; ++i)
          for (int j = i + 1; j < 3; ++j) {
            if (m->noncompact) {
              const double F = nc_F(m, L, i, j, s);
              acc[5] += F * F;
            } else {
              acc[5] += 1.0 - plaquette(m, L, i, j, s).re;
            }
          }
        acc[6] += p.re;
        acc[7] += p.im;
        acc[8] += r2;
      }
  }
  for (int k = 0; k < nacc; ++k) {
    double sacc = 0.0;
    for (int x = 0; x < N; ++x) sacc += part[(size_t)x * nacc + k];
    out[k] = sacc / (double)V;
  }
  free(part);
}

/* Energies (Sec. 5.4.1): e[0] = E_K^phi = <|pi|^2>/a^6, e[1] = E_G^phi = <sum|D+phi|^2>/a^2,
   e[2] = E_V, e[3] = E_K^A = (w_star/f_star)^2 sum <piA^2>/(2 a^4),
   e[4] = E_G^A = (w_star/f_star)^2 /(a^4 dx^4 e^2) sum_{i<j} <1 - Re V_ij>
          (non-compact: (w_star/f_star)^2 /(2 a^4) sum_{i<j} <F_ij^2>, Sec. 5.2 read with
          F_ij = D+_i A_j - D+_j A_i),
   e[5] = <lambda|phi|^4>, e[6] = <m2|phi|^2>.  kin_phi / kin_A override the kinetic
   averages when >= 0 (staggered averages). */
static void u1_energies(const orc_u1* m, double a, const double* s, double kin_phi, double kin_A, double* e) {
  const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2, dx2 = m->dx * m->dx;
  e[0] = (kin_phi >= 0.0 ? kin_phi : s[0]) / a6;
  e[1] = s[1] / (a2 * dx2);
  e[2] = s[2] + s[3];
  e[3] = m->wf2 * (kin_A >= 0.0 ? kin_A : s[4]) / (2.0 * a4);
  e[4] = m->noncompact ? m->wf2 * s[5] / (2.0 * a4) : m->wf2 * s[5] / (a4 * dx2 * dx2 * m->e * m->e);
  e[5] = s[2];
  e[6] = s[3];
}

/* Scale-factor kernel with the gauge term (Sec. 5.1):
   K_a = (1/3)(f/m_p)^2 a^{1+2 alpha} [(alpha-2) E_K^phi + alpha E_G^phi + (alpha+1) E_V
                                        + (alpha-1)(E_K^A + E_G^A)] */
double orc_u1_Ka(const orc_u1* m, double a, const double* e) {
  const double al = m->alpha;
  return m->fmp2 / 3.0 * pow(a, 1.0 + 2.0 * al) *
         ((al - 2.0) * e[0] + al * e[1] + (al + 1.0) * e[2] + (al - 1.0) * (e[3] + e[4]));
}

/* Cayley link drift (Sec. 5.3, drift from momenta, exact form):
   V <- (1 - i u)/(1 + i u) V,  u = e h dx piA / (2 a_mid^{1-alpha}). */
static void u1_link_drift(const orc_u1* m, double* L, const double* piA, double h, double amid) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  if (m->noncompact) {
    /* A_i += h piA_i / a_mid^{1-alpha} (Sec. 5.2) */
    const double cA = h / pow(amid, 1.0 - m->alpha);
    for (int64_t k = 0; k < 3 * V; ++k) L[k] += cA * piA[k];
    return;
  }
  const double c = m->e * h * m->dx / (2.0 * pow(amid, 1.0 - m->alpha));
  for (int i = 0; i < 3; ++i)
    for (int64_t s = 0; s < V; ++s) {
      const double u = c * piA[i * V + s];
      const double d = 1.0 + u * u;
      const cpx r = cmk((1.0 - u * u) / d, -2.0 * u / d);
      const cpx v = cmul_(r, link_c(L, V, i, s));
      L[(2 * i) * V + s] = v.re;
      L[(2 * i + 1) * V + s] = v.im;
    }
}

static double sum_sq(const double* x, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += x[i] * x[i];
  return s;
}

/* Start-up of the staggered leapfrog from a synchronised state:
   pi_{-1/2} = pi_0 - (h/2) K_phi, piA_{-1/2} = piA_0 - (h/2) K_A,
   b_{-1/2} = b_0 - (h/2) K_a[a_0, E(synchronised)]. */
void orc_u1_lf_startup(const orc_u1* m, double* phi, double* pi, double* L, double* piA, double* a, double* b,
                       double h) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* Kp = (double*)malloc(sizeof(double) * 2 * V);
  double* KA = (double*)malloc(sizeof(double) * 3 * V);
  double s[9], e[7];
  if (m->expand) {
    orc_u1_sums(m, phi, pi, L, piA, s);
    u1_energies(m, *a, s, -1.0, -1.0, e);
    *b = *b - 0.5 * h * orc_u1_Ka(m, *a, e);
  }
  orc_u1_kernels(m, *a, phi, L, Kp, KA);
  for (int64_t i = 0; i < 2 * V; ++i) pi[i] -= 0.5 * h * Kp[i];
  for (int64_t i = 0; i < 3 * V; ++i) piA[i] -= 0.5 * h * KA[i];
  free(Kp);
  free(KA);
}

/* Compact staggered leapfrog (Sec. 5.3.1), per step:
     pi_{+1/2}  = pi_{-1/2} + h K_phi[a, phi, V]
     piA_{+1/2} = piA_{-1/2} + h K_A[a, phi, V]
     b_{+1/2}   = b_{-1/2} + h K_a[a, avg E_K^phi, E_G^phi, E_V, avg E_K^A, E_G^A]
     a_{+1}     = a + h b_{+1/2}
     phi_{+1}   = phi + h pi_{+1/2} / a_{+1/2}^{3-alpha}
     V_{+1}     = Cayley(piA_{+1/2}) V
   The kinetic averages take both staggered momenta with the scale factor at n. */
void orc_u1_lf_steps(const orc_u1* m, double* phi, double* pi, double* L, double* piA, double* a, double* b,
                     double h, int64_t nsteps) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* Kp = (double*)malloc(sizeof(double) * 2 * V);
  double* KA = (double*)malloc(sizeof(double) * 3 * V);
  double s[9], e[7];
  for (int64_t it = 0; it < nsteps; ++it) {
    orc_u1_kernels(m, *a, phi, L, Kp, KA);
    const double kp0 = sum_sq(pi, 2 * V), ka0 = sum_sq(piA, 3 * V);
    for (int64_t i = 0; i < 2 * V; ++i) pi[i] += h * Kp[i];
    for (int64_t i = 0; i < 3 * V; ++i) piA[i] += h * KA[i];
    double anew = *a, amid = *a;
    if (m->expand) {
      const double kp1 = sum_sq(pi, 2 * V), ka1 = sum_sq(piA, 3 * V);
      orc_u1_sums(m, phi, NULL, L, NULL, s);
      u1_energies(m, *a, s, 0.5 * (kp0 + kp1) / (double)V, 0.5 * (ka0 + ka1) / (double)V, e);
      *b = *b + h * orc_u1_Ka(m, *a, e);
      anew = *a + h * (*b);
      amid = 0.5 * (*a + anew);
    }
    const double cd = h * pow(amid, -(3.0 - m->alpha));
    for (int64_t i = 0; i < 2 * V; ++i) phi[i] += cd * pi[i];
    u1_link_drift(m, L, piA, h, amid);
    *a = anew;
  }
  free(Kp);
  free(KA);
}

/* Compact velocity Verlet (Sec. 5.3.2) and its Yoshida compositions
   (Sec. 5.3.3): for each sub-step weight w, with hw = w h,
     b   += (hw/2) K_a[a, E(phi, pi, V, piA)]
     pi  += (hw/2) K_phi[a, phi, V],   piA += (hw/2) K_A[a, phi, V]
     a'   = a + hw b,  a_mid = (a + a')/2
     phi += hw pi / a_mid^{3-alpha},   V = Cayley(hw, piA, a_mid) V,   a = a'
     pi  += (hw/2) K_phi[a, phi, V],   piA += (hw/2) K_A[a, phi, V]
     b   += (hw/2) K_a[a, E(phi, pi, V, piA)]
   (the same order as the scalar scheme, orc_vv_substep). */
void orc_u1_vv_steps(const orc_u1* m, double* phi, double* pi, double* L, double* piA, double* a, double* b,
                     double h, const double* w, int nw, int64_t nsteps) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* Kp = (double*)malloc(sizeof(double) * 2 * V);
  double* KA = (double*)malloc(sizeof(double) * 3 * V);
  double s[9], e[7];
  for (int64_t it = 0; it < nsteps; ++it) {
    for (int p = 0; p < nw; ++p) {
      const double hw = w[p] * h;
      if (m->expand) {
        orc_u1_sums(m, phi, pi, L, piA, s);
        u1_energies(m, *a, s, -1.0, -1.0, e);
        *b += 0.5 * hw * orc_u1_Ka(m, *a, e);
      }
      orc_u1_kernels(m, *a, phi, L, Kp, KA);
      for (int64_t i = 0; i < 2 * V; ++i) pi[i] += 0.5 * hw * Kp[i];
      for (int64_t i = 0; i < 3 * V; ++i) piA[i] += 0.5 * hw * KA[i];
      double anew = *a, amid = *a;
      if (m->expand) {
        anew = *a + hw * (*b);
        amid = 0.5 * (*a + anew);
      }
      const double cd = hw * pow(amid, -(3.0 - m->alpha));
      for (int64_t i = 0; i < 2 * V; ++i) phi[i] += cd * pi[i];
      u1_link_drift(m, L, piA, hw, amid);
      *a = anew;
      orc_u1_kernels(m, *a, phi, L, Kp, KA);
      for (int64_t i = 0; i < 2 * V; ++i) pi[i] += 0.5 * hw * Kp[i];
      for (int64_t i = 0; i < 3 * V; ++i) piA[i] += 0.5 * hw * KA[i];
      if (m->expand) {
        orc_u1_sums(m, phi, pi, L, piA, s);
        u1_energies(m, *a, s, -1.0, -1.0, e);
        *b += 0.5 * hw * orc_u1_Ka(m, *a, e);
      }
    }
  }
  free(Kp);
  free(KA);
}

/* Gauss-law residual (Sec. 5.2 discrete Gauss law, sign fixed by the kick):
   G(n) = sum_i (piA_i(n) - piA_i(n-i))/dx - 2 e (f_star/w_star)^2 Im[conj phi(n) pi(n)];
   out[0] = sum G^2, out[1] = sum (div piA)^2, out[2] = sum rho^2, out[3] = sum rho. */
void orc_u1_gauss(const orc_u1* m, const double* phi, const double* pi, const double* piA, double* out) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  double g2 = 0.0, d2 = 0.0, r2 = 0.0, rs = 0.0;
  for (int64_t s = 0; s < V; ++s) {
    double div = 0.0;
    for (int i = 0; i < 3; ++i) div += (piA[i * V + s] - piA[i * V + shift(N, s, i, -1)]) / m->dx;
    const double rho = 2.0 * m->e / m->wf2 * (phi[s] * pi[V + s] - phi[V + s] * pi[s]);
    g2 += (div - rho) * (div - rho);
    d2 += div * div;
    r2 += rho * rho;
    rs += rho;
  }
  out[0] = g2;
  out[1] = d2;
  out[2] = r2;
  out[3] = rs;
}

/* Observables of a staggered state (phi_n, V_n, a_n; pi_{n-1/2}, piA_{n-1/2}, b_{n-1/2}):
   e[0..6] as u1_energies with the averaged kinetic terms, e[7] = b_n (mean of the two
   half-step values), e[8] = Hubble-constraint residual, e[9] = Gauss residual
   ||G|| / (||div piA|| + ||rho||) of the stored half-step momenta,
   e[10..12] = <Re phi>, <Im phi>, <|phi|^2>. */
void orc_u1_lf_observe(const orc_u1* m, const double* phi, const double* pi, const double* L, const double* piA,
                       double a, double b, double h, double* e) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* Kp = (double*)malloc(sizeof(double) * 2 * V);
  double* KA = (double*)malloc(sizeof(double) * 3 * V);
  orc_u1_kernels(m, a, phi, L, Kp, KA);
  double kp1 = 0.0, ka1 = 0.0;
  for (int64_t i = 0; i < 2 * V; ++i) { const double v = pi[i] + h * Kp[i]; kp1 += v * v; }
  for (int64_t i = 0; i < 3 * V; ++i) { const double v = piA[i] + h * KA[i]; ka1 += v * v; }
  const double kp0 = sum_sq(pi, 2 * V), ka0 = sum_sq(piA, 3 * V);
  double s[9];
  orc_u1_sums(m, phi, NULL, L, NULL, s);
  u1_energies(m, a, s, 0.5 * (kp0 + kp1) / (double)V, 0.5 * (ka0 + ka1) / (double)V, e);
  double bn = b, hc = 0.0;
  if (m->expand) {
    const double bp = b + h * orc_u1_Ka(m, a, e);
    bn = 0.5 * (b + bp);
    const double rho = e[0] + e[1] + e[2] + e[3] + e[4];
    const double rhs = m->fmp2 / 3.0 * pow(a, 2.0 * (m->alpha + 1.0)) * rho;
    hc = fabs(bn * bn - rhs) / (bn * bn);
  }
  double g[4];
  orc_u1_gauss(m, phi, pi, piA, g);
  e[7] = bn;
  e[8] = hc;
  e[9] = sqrt(g[0]) / (sqrt(g[1]) + sqrt(g[2]));
  e[10] = s[6];
  e[11] = s[7];
  e[12] = s[8];
  free(Kp);
  free(KA);
}

/* Observables of a synchronised state; same layout as orc_u1_lf_observe. */
void orc_u1_sync_observe(const orc_u1* m, const double* phi, const double* pi, const double* L,
                         const double* piA, double a, double b, double* e) {
  double s[9];
  orc_u1_sums(m, phi, pi, L, piA, s);
  u1_energies(m, a, s, -1.0, -1.0, e);
  double hc = 0.0;
  if (m->expand) {
    const double rho = e[0] + e[1] + e[2] + e[3] + e[4];
    const double rhs = m->fmp2 / 3.0 * pow(a, 2.0 * (m->alpha + 1.0)) * rho;
    hc = fabs(b * b - rhs) / (b * b);
  }
  double g[4];
  orc_u1_gauss(m, phi, pi, piA, g);
  e[7] = b;
  e[8] = hc;
  e[9] = sqrt(g[0]) / (sqrt(g[1]) + sqrt(g[2]));
  e[10] = s[6];
  e[11] = s[7];
  e[12] = s[8];
}

/* ------------------------------------------------------------------ */
/* Doublet with SU(2) x U(1) gauge links (Sec. 6; SU(N) toolkit of     */
/* Sec. 3.2.2).  Phi = (Phi_0, Phi_1), Phi_c = (phi_2c + i phi_2c+1)    */
/* /sqrt 2, stored as four reals (Re Phi_0, Im Phi_0, Re Phi_1,        */
/* Im Phi_1).  U(1) link V_i = exp(i th_i) stored (Re, Im); SU(2) link  */
/* U_i = c0 + i c.sigma stored (c0, c1, c2, c3), in matrix form        */
/*   [[c0 + i c3, c2 + i c1], [-c2 + i c1, c0 - i c3]].                */
/* pi_A,i: one real per link; pi_B,i: three reals per link, the        */
/* components along T_a = sigma_a/2.  The equations are those of the   */
/* lattice Hamiltonian whose energies the paper lists (Sec. 6.3.1):    */
/*   E_K^Phi = <pi^dag pi>/a^6, E_G^Phi = sum_i <|V_i U_i Phi_{+i}     */
/*   - Phi|^2>/(a^2 dx^2), E_K^B = (w/f)^2 sum <pi_B^2>/(2 a^4),        */
/*   E_G^B = 2 (w/f)^2/(a^4 dx^4 g^2) sum_{i<j} <2 - Tr U_ij>,          */
/* with U(1) as in Sec. 5; the electric fields generate left          */
/* multiplication of the links (U' = -i g dx pi_B U / a^{1-alpha},      */
/* Sec. 6.2), so each force is minus the derivative of the energy     */
/* along that motion.  Arithmetic: explicit 2x2 complex matrices.      */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t N, expand, pad0, pad1;
  double dx, alpha, fmp2;
  double lambda;   /* V = lambda |Phi|^4 + m2 |Phi|^2, |Phi|^2 = Phi^dag Phi */
  double m2;
  double e;        /* U(1) coupling of the doublet, g_A Q_A */
  double g;        /* SU(2) coupling, g_B Q_B */
  double wf2;      /* (w_star/f_star)^2 */
} orc_su2;

typedef struct { cpx m[2][2]; } mat2;

static mat2 mat_of_c(double c0, double c1, double c2, double c3) {
  mat2 r;
  r.m[0][0] = cmk(c0, c3);
  r.m[0][1] = cmk(c2, c1);
  r.m[1][0] = cmk(-c2, c1);
  r.m[1][1] = cmk(c0, -c3);
  return r;
}
static mat2 mat_mul(mat2 a, mat2 b) {
  mat2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const cpx p = cmul_(a.m[i][0], b.m[0][j]), q = cmul_(a.m[i][1], b.m[1][j]);
      r.m[i][j] = cmk(p.re + q.re, p.im + q.im);
    }
  return r;
}
static mat2 mat_dag(mat2 a) {
  mat2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.m[i][j] = cconj_(a.m[j][i]);
  return r;
}
static mat2 mat_scale(mat2 a, cpx s) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) a.m[i][j] = cmul_(s, a.m[i][j]);
  return a;
}
/* Pauli matrices sigma_1..3 */
static mat2 pauli(int a) {
  mat2 r;
  r.m[0][0] = r.m[0][1] = r.m[1][0] = r.m[1][1] = cmk(0.0, 0.0);
  if (a == 1) { r.m[0][1] = cmk(1.0, 0.0); r.m[1][0] = cmk(1.0, 0.0); }
  else if (a == 2) { r.m[0][1] = cmk(0.0, -1.0); r.m[1][0] = cmk(0.0, 1.0); }
  else { r.m[0][0] = cmk(1.0, 0.0); r.m[1][1] = cmk(-1.0, 0.0); }
  return r;
}
static cpx mat_trace(mat2 a) { return cmk(a.m[0][0].re + a.m[1][1].re, a.m[0][0].im + a.m[1][1].im); }
/* c_a of an SU(2) element M = c0 + i c.sigma: Tr(sigma_a M) = 2 i c_a */
static double su2_coef(mat2 M, int a) { return 0.5 * mat_trace(mat_mul(pauli(a), M)).im; }
/* matrix of the algebra element sum_a x^a T_a, T_a = sigma_a/2 */
static mat2 alg_mat(const double x[3]) {
  mat2 r;
  r.m[0][0] = cmk(0.5 * x[2], 0.0);
  r.m[0][1] = cmk(0.5 * x[0], -0.5 * x[1]);
  r.m[1][0] = cmk(0.5 * x[0], 0.5 * x[1]);
  r.m[1][1] = cmk(-0.5 * x[2], 0.0);
  return r;
}
/* components x^a of a Hermitian traceless X = x^a T_a: x^a = Tr(sigma_a X) */
static void alg_comp(mat2 X, double x[3]) {
  for (int a = 1; a <= 3; ++a) x[a - 1] = mat_trace(mat_mul(pauli(a), X)).re;
}

typedef struct { cpx v[2]; } vec2;
static vec2 mat_vec(mat2 A, vec2 x) {
  vec2 r;
  for (int i = 0; i < 2; ++i) {
    const cpx p = cmul_(A.m[i][0], x.v[0]), q = cmul_(A.m[i][1], x.v[1]);
    r.v[i] = cmk(p.re + q.re, p.im + q.im);
  }
  return r;
}
/* x^dag y */
static cpx vdot(vec2 x, vec2 y) {
  const cpx p = cmul_(cconj_(x.v[0]), y.v[0]), q = cmul_(cconj_(x.v[1]), y.v[1]);
  return cmk(p.re + q.re, p.im + q.im);
}

static vec2 dbl_at(const double* phi, int64_t V, int64_t s) {
  vec2 r;
  r.v[0] = cmk(phi[s], phi[V + s]);
  r.v[1] = cmk(phi[2 * V + s], phi[3 * V + s]);
  return r;
}
static mat2 su2_link(const double* UL, int64_t V, int i, int64_t s) {
  const double* b = UL + (size_t)4 * i * V;
  return mat_of_c(b[s], b[V + s], b[2 * V + s], b[3 * V + s]);
}
/* W_i(n) = V_i(n) U_i(n), the combined link acting on the doublet */
static mat2 dbl_link(const double* VL, const double* UL, int64_t V, int i, int64_t s) {
  return mat_scale(su2_link(UL, V, i, s), link_c(VL, V, i, s));
}
static mat2 su2_plaquette(const orc_su2* m, const double* UL, int i, int j, int64_t s) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  return mat_mul(mat_mul(su2_link(UL, V, i, s), su2_link(UL, V, j, shift(N, s, i, 1))),
                 mat_mul(mat_dag(su2_link(UL, V, i, shift(N, s, j, 1))), mat_dag(su2_link(UL, V, j, s))));
}
static cpx u1_plaquette_c(const orc_su2* m, const double* VL, int i, int j, int64_t s) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  const cpx a = link_c(VL, V, i, s), b = link_c(VL, V, j, shift(N, s, i, 1));
  const cpx c = cconj_(link_c(VL, V, i, shift(N, s, j, 1))), d = cconj_(link_c(VL, V, j, s));
  return cmul_(cmul_(a, b), cmul_(c, d));
}

/* Kernels (Sec. 6.2, written as the forces of the energies above):
   K_Phi    = a^{1+alpha} sum_i (W_i Phi_{+i} - 2 Phi + W_i(n-i)^dag Phi_{-i}) / dx^2
              - a^{3+alpha} (2 lambda |Phi|^2 + m2) Phi
   K_A,i    = a^{1+alpha} (2e/dx)(f/w)^2 Im[Phi^dag W_i Phi_{+i}]
              + a^{alpha-1}/(e dx^3) sum_{j!=i} (Im V_ij(n) - Im V_ij(n-j))
   K_B,i^a  = a^{1+alpha} (g/dx)(f/w)^2 Im[Phi^dag sigma_a W_i Phi_{+i}]
              + a^{alpha-1} 2/(g dx^3) sum_{j!=i} (c_a[U_ij(n)] - c_a[U_j(n-j)^dag U_ij(n-j) U_j(n-j)]) */
void orc_su2_kernels(const orc_su2* m, double a, const double* phi, const double* VL, const double* UL,
                     double* Kphi, double* KA, double* KB) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  const double cl = pow(a, 1.0 + m->alpha) / (m->dx * m->dx);
  const double cp = pow(a, 3.0 + m->alpha);
  const double cjA = pow(a, 1.0 + m->alpha) * 2.0 * m->e / m->dx / m->wf2;
  const double cjB = pow(a, 1.0 + m->alpha) * m->g / m->dx / m->wf2;
  const double cbA = pow(a, m->alpha - 1.0) / (m->e * m->dx * m->dx * m->dx);
  const double cbB = pow(a, m->alpha - 1.0) * 2.0 / (m->g * m->dx * m->dx * m->dx);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < N; ++x)
    for (int y = 0; y < N; ++y)
      for (int z = 0; z < N; ++z) {
        const int64_t s = site(N, x, y, z);
        const vec2 p = dbl_at(phi, V, s);
        vec2 lap;
        for (int c = 0; c < 2; ++c) lap.v[c] = cmk(-6.0 * p.v[c].re, -6.0 * p.v[c].im);
        vec2 fw[3];
        for (int i = 0; i < 3; ++i) {
          const int64_t sp = shift(N, s, i, 1), sm = shift(N, s, i, -1);
          fw[i] = mat_vec(dbl_link(VL, UL, V, i, s), dbl_at(phi, V, sp));
          const vec2 bw = mat_vec(mat_dag(dbl_link(VL, UL, V, i, sm)), dbl_at(phi, V, sm));
          for (int c = 0; c < 2; ++c) {
            lap.v[c].re += fw[i].v[c].re + bw.v[c].re;
            lap.v[c].im += fw[i].v[c].im + bw.v[c].im;
          }
        }
        const double r2 = vdot(p, p).re;
        const double dv = 2.0 * m->lambda * r2 + m->m2;
        for (int c = 0; c < 2; ++c) {
          Kphi[(2 * c) * V + s] = cl * lap.v[c].re - cp * dv * p.v[c].re;
          Kphi[(2 * c + 1) * V + s] = cl * lap.v[c].im - cp * dv * p.v[c].im;
        }
        for (int i = 0; i < 3; ++i) {
          double magA = 0.0, magB[3] = {0.0, 0.0, 0.0};
          for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            const int64_t sjm = shift(N, s, j, -1);
            magA += u1_plaquette_c(m, VL, i, j, s).im - u1_plaquette_c(m, VL, i, j, sjm).im;
            const mat2 Pn = su2_plaquette(m, UL, i, j, s);
            const mat2 Uj = su2_link(UL, V, j, sjm);
            const mat2 Pm = mat_mul(mat_mul(mat_dag(Uj), su2_plaquette(m, UL, i, j, sjm)), Uj);
            for (int a = 1; a <= 3; ++a) magB[a - 1] += su2_coef(Pn, a) - su2_coef(Pm, a);
          }
          KA[i * V + s] = cjA * vdot(p, fw[i]).im + cbA * magA;
          for (int a = 1; a <= 3; ++a)
            KB[(3 * i + a - 1) * V + s] = cjB * vdot(p, mat_vec(pauli(a), fw[i])).im + cbB * magB[a - 1];
        }
      }
}

/* Raw volume averages: out[0] = <pi^dag pi>, out[1] = <sum_i |W_i Phi_{+i} - Phi|^2>,
   out[2] = <lambda |Phi|^4>, out[3] = <m2 |Phi|^2>, out[4] = <sum_i piA_i^2>,
   out[5] = <sum_{i<j} (1 - Re V_ij)>, out[6] = <sum_{i,a} piB_i^a^2>, out[7] = <sum_{i<j} (2 - Tr U_ij)>,
   out[8..11] = <the four real components of Phi>, out[12] = <|Phi|^2>. */
#define ORC_SU2_NS 13
void orc_su2_sums(const orc_su2* m, const double* phi, const double* pi, const double* VL, const double* UL,
                  const double* piA, const double* piB, double* out) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  double* part = (double*)calloc((size_t)N * ORC_SU2_NS, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int x = 0; x < N; ++x) {
    double* acc = part + (size_t)x * ORC_SU2_NS;
    for (int y = 0; y < N; ++y)
      for (int z = 0; z < N; ++z) {
        const int64_t s = site(N, x, y, z);
        const vec2 p = dbl_at(phi, V, s);
        if (pi)
          for (int k = 0; k < 4; ++k) acc[0] += pi[k * V + s] * pi[k * V + s];
        for (int i = 0; i < 3; ++i) {
          const vec2 f = mat_vec(dbl_link(VL, UL, V, i, s), dbl_at(phi, V, shift(N, s, i, 1)));
          for (int c = 0; c < 2; ++c) {
            const double dr = f.v[c].re - p.v[c].re, di = f.v[c].im - p.v[c].im;
            acc[1] += dr * dr + di * di;
          }
          if (piA) acc[4] += piA[i * V + s] * piA[i * V + s];
          if (piB)
            for (int a = 0; a < 3; ++a) acc[6] += piB[(3 * i + a) * V + s] * piB[(3 * i + a) * V + s];
        }
        const double r2 = vdot(p, p).re;
        acc[2] += m->lambda * r2 * r2;
        acc[3] += m->m2 * r2;
        for (int i = 0; i < 3; ++i)
          for (int j = i + 1; j < 3; ++j) {
            acc[5] += 1.0 - u1_plaquette_c(m, VL, i, j, s).re;
            acc[7] += 2.0 - mat_trace(su2_plaquette(m, UL, i, j, s)).re;
          }
        for (int k = 0; k < 4; ++k) acc[8 + k] += phi[k * V + s];
        acc[12] += r2;
      }
  }
  for (int k = 0; k < ORC_SU2_NS; ++k) {
    double sacc = 0.0;
    for (int x = 0; x < N; ++x) sacc += part[(size_t)x * ORC_SU2_NS + k];
    out[k] = sacc / (double)V;
  }
  free(part);
}

/* Energies: e[0] E_K^Phi, e[1] E_G^Phi, e[2] E_V, e[3] E_K^A, e[4] E_G^A, e[5] E_K^B, e[6] E_G^B,
   e[7] <lambda|Phi|^4>, e[8] <m2|Phi|^2>.  kin_* >= 0 override the kinetic averages. */
static void su2_energies(const orc_su2* m, double a, const double* s, double kin_phi, double kin_A, double kin_B,
                         double* e) {
  const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2, dx2 = m->dx * m->dx, dx4 = dx2 * dx2;
  e[0] = (kin_phi >= 0.0 ? kin_phi : s[0]) / a6;
  e[1] = s[1] / (a2 * dx2);
  e[2] = s[2] + s[3];
  e[3] = m->wf2 * (kin_A >= 0.0 ? kin_A : s[4]) / (2.0 * a4);
  e[4] = m->wf2 * s[5] / (a4 * dx4 * m->e * m->e);
  e[5] = m->wf2 * (kin_B >= 0.0 ? kin_B : s[6]) / (2.0 * a4);
  e[6] = 2.0 * m->wf2 * s[7] / (a4 * dx4 * m->g * m->g);
  e[7] = s[2];
  e[8] = s[3];
}

/* K_a with both gauge sectors, radiation-like: (alpha-1)(E_K^A + E_G^A + E_K^B + E_G^B) */
double orc_su2_Ka(const orc_su2* m, double a, const double* e) {
  const double al = m->alpha;
  return m->fmp2 / 3.0 * pow(a, 1.0 + 2.0 * al) *
         ((al - 2.0) * e[0] + al * e[1] + (al + 1.0) * e[2] + (al - 1.0) * (e[3] + e[4] + e[5] + e[6]));
}

/* Link drifts (Sec. 6.2 drift from momenta, Cayley form):
   V <- (1 - i u)/(1 + i u) V,   u = e h dx piA / (2 a_mid^{1-alpha});
   U <- (1 - i X)(1 + i X)^{-1} U, X = w^a sigma_a, w^a = g h dx piB^a / (4 a_mid^{1-alpha})
   (the Cayley transform of -i g h dx piB^a T_a / a_mid^{1-alpha}; unitary, det 1). */
static void su2_link_drift(const orc_su2* m, double* VL, double* UL, const double* piA, const double* piB, double h,
                           double amid) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  const double cA = m->e * h * m->dx / (2.0 * pow(amid, 1.0 - m->alpha));
  const double cB = m->g * h * m->dx / (4.0 * pow(amid, 1.0 - m->alpha));
  for (int i = 0; i < 3; ++i)
    for (int64_t s = 0; s < V; ++s) {
      const double u = cA * piA[i * V + s];
      const double d = 1.0 + u * u;
      const cpx r = cmk((1.0 - u * u) / d, -2.0 * u / d);
      const cpx v = cmul_(r, link_c(VL, V, i, s));
      VL[(2 * i) * V + s] = v.re;
      VL[(2 * i + 1) * V + s] = v.im;
      /* (1 - iX)(1 + iX)^{-1} = (1 - iX)^2 / (1 + |w|^2) since X^2 = |w|^2 */
      double w[3];
      for (int a = 0; a < 3; ++a) w[a] = cB * piB[(3 * i + a) * V + s];
      const double w2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
      const mat2 C = mat_of_c((1.0 - w2) / (1.0 + w2), -2.0 * w[0] / (1.0 + w2), -2.0 * w[1] / (1.0 + w2),
                              -2.0 * w[2] / (1.0 + w2));
      const mat2 Un = mat_mul(C, su2_link(UL, V, i, s));
      double* b = UL + (size_t)4 * i * V;
      b[s] = Un.m[0][0].re;
      b[V + s] = Un.m[0][1].im;
      b[2 * V + s] = Un.m[0][1].re;
      b[3 * V + s] = Un.m[0][0].im;
    }
}

/* Start-up of the staggered leapfrog from a synchronised state (as orc_u1_lf_startup). */
void orc_su2_lf_startup(const orc_su2* m, double* phi, double* pi, double* VL, double* UL, double* piA,
                        double* piB, double* a, double* b, double h) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* Kp = (double*)malloc(sizeof(double) * 4 * V);
  double* KA = (double*)malloc(sizeof(double) * 3 * V);
  double* KB = (double*)malloc(sizeof(double) * 9 * V);
  double s[ORC_SU2_NS], e[9];
  if (m->expand) {
    orc_su2_sums(m, phi, pi, VL, UL, piA, piB, s);
    su2_energies(m, *a, s, -1.0, -1.0, -1.0, e);
    *b = *b - 0.5 * h * orc_su2_Ka(m, *a, e);
  }
  orc_su2_kernels(m, *a, phi, VL, UL, Kp, KA, KB);
  for (int64_t i = 0; i < 4 * V; ++i) pi[i] -= 0.5 * h * Kp[i];
  for (int64_t i = 0; i < 3 * V; ++i) piA[i] -= 0.5 * h * KA[i];
  for (int64_t i = 0; i < 9 * V; ++i) piB[i] -= 0.5 * h * KB[i];
  free(Kp);
  free(KA);
  free(KB);
}

/* SU(N) staggered leapfrog (Sec. 6.2.1), per step:
     pi_{+1/2} = pi_{-1/2} + h K_Phi;  piA, piB likewise
     b_{+1/2}  = b_{-1/2} + h K_a[a, semi-sums of the kinetic energies, E_G, E_V]
     a_{+1}    = a + h b_{+1/2};  Phi += h pi_{+1/2} / a_{+1/2}^{3-alpha};  links drifted */
void orc_su2_lf_steps(const orc_su2* m, double* phi, double* pi, double* VL, double* UL, double* piA, double* piB,
                      double* a, double* b, double h, int64_t nsteps) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* Kp = (double*)malloc(sizeof(double) * 4 * V);
  double* KA = (double*)malloc(sizeof(double) * 3 * V);
  double* KB = (double*)malloc(sizeof(double) * 9 * V);
  double s[ORC_SU2_NS], e[9];
  for (int64_t it = 0; it < nsteps; ++it) {
    orc_su2_kernels(m, *a, phi, VL, UL, Kp, KA, KB);
    const double kp0 = sum_sq(pi, 4 * V), ka0 = sum_sq(piA, 3 * V), kb0 = sum_sq(piB, 9 * V);
    for (int64_t i = 0; i < 4 * V; ++i) pi[i] += h * Kp[i];
    for (int64_t i = 0; i < 3 * V; ++i) piA[i] += h * KA[i];
    for (int64_t i = 0; i < 9 * V; ++i) piB[i] += h * KB[i];
    double anew = *a, amid = *a;
    if (m->expand) {
      const double kp1 = sum_sq(pi, 4 * V), ka1 = sum_sq(piA, 3 * V), kb1 = sum_sq(piB, 9 * V);
      orc_su2_sums(m, phi, NULL, VL, UL, NULL, NULL, s);
      su2_energies(m, *a, s, 0.5 * (kp0 + kp1) / (double)V, 0.5 * (ka0 + ka1) / (double)V,
                   0.5 * (kb0 + kb1) / (double)V, e);
      *b = *b + h * orc_su2_Ka(m, *a, e);
      anew = *a + h * (*b);
      amid = 0.5 * (*a + anew);
    }
    const double cd = h * pow(amid, -(3.0 - m->alpha));
    for (int64_t i = 0; i < 4 * V; ++i) phi[i] += cd * pi[i];
    su2_link_drift(m, VL, UL, piA, piB, h, amid);
    *a = anew;
  }
  free(Kp);
  free(KA);
  free(KB);
}

/* Velocity Verlet and its Yoshida compositions (Sec. 6.2.2, 6.2.3), in the
   order of orc_u1_vv_steps. */
void orc_su2_vv_steps(const orc_su2* m, double* phi, double* pi, double* VL, double* UL, double* piA, double* piB,
                      double* a, double* b, double h, const double* w, int nw, int64_t nsteps) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double* Kp = (double*)malloc(sizeof(double) * 4 * V);
  double* KA = (double*)malloc(sizeof(double) * 3 * V);
  double* KB = (double*)malloc(sizeof(double) * 9 * V);
  double s[ORC_SU2_NS], e[9];
  for (int64_t it = 0; it < nsteps; ++it) {
    for (int p = 0; p < nw; ++p) {
      const double hw = w[p] * h;
      if (m->expand) {
        orc_su2_sums(m, phi, pi, VL, UL, piA, piB, s);
        su2_energies(m, *a, s, -1.0, -1.0, -1.0, e);
        *b += 0.5 * hw * orc_su2_Ka(m, *a, e);
      }
      orc_su2_kernels(m, *a, phi, VL, UL, Kp, KA, KB);
      for (int64_t i = 0; i < 4 * V; ++i) pi[i] += 0.5 * hw * Kp[i];
      for (int64_t i = 0; i < 3 * V; ++i) piA[i] += 0.5 * hw * KA[i];
      for (int64_t i = 0; i < 9 * V; ++i) piB[i] += 0.5 * hw * KB[i];
      double anew = *a, amid = *a;
      if (m->expand) {
        anew = *a + hw * (*b);
        amid = 0.5 * (*a + anew);
      }
      const double cd = hw * pow(amid, -(3.0 - m->alpha));
      for (int64_t i = 0; i < 4 * V; ++i) phi[i] += cd * pi[i];
      su2_link_drift(m, VL, UL, piA, piB, hw, amid);
      *a = anew;
      orc_su2_kernels(m, *a, phi, VL, UL, Kp, KA, KB);
      for (int64_t i = 0; i < 4 * V; ++i) pi[i] += 0.5 * hw * Kp[i];
      for (int64_t i = 0; i < 3 * V; ++i) piA[i] += 0.5 * hw * KA[i];
      for (int64_t i = 0; i < 9 * V; ++i) piB[i] += 0.5 * hw * KB[i];
      if (m->expand) {
        orc_su2_sums(m, phi, pi, VL, UL, piA, piB, s);
        su2_energies(m, *a, s, -1.0, -1.0, -1.0, e);
        *b += 0.5 * hw * orc_su2_Ka(m, *a, e);
      }
    }
  }
  free(Kp);
  free(KA);
  free(KB);
}

/* Gauss residuals (Sec. 5.2 for U(1); Sec. 6.2, discrete SU(N) Gauss law with the
   electric field at n - i parallel-transported to n):
   G_A(n)   = sum_i (piA_i(n) - piA_i(n-i))/dx - 2e (f/w)^2 Im[Phi^dag pi]
   G_B^a(n) = sum_i (piB_i(n) - U_i(n-i)^dag piB_i(n-i) U_i(n-i))^a / dx - g (f/w)^2 Im[Phi^dag sigma_a pi]
   out[0..2] = sum G_A^2, sum div_A^2, sum rho_A^2; out[3..5] the same for SU(2) (over a);
   out[6] = sum rho_A, out[7..9] = sum rho_B^a. */
void orc_su2_gauss(const orc_su2* m, const double* phi, const double* pi, const double* UL, const double* piA,
                   const double* piB, double* out) {
  const int N = m->N;
  const int64_t V = (int64_t)N * N * N;
  for (int k = 0; k < 10; ++k) out[k] = 0.0;
  for (int64_t s = 0; s < V; ++s) {
    const vec2 p = dbl_at(phi, V, s), q = dbl_at(pi, V, s);
    double divA = 0.0, divB[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) {
      const int64_t sm = shift(N, s, i, -1);
      divA += (piA[i * V + s] - piA[i * V + sm]) / m->dx;
      double xm[3], xt[3];
      for (int a = 0; a < 3; ++a) xm[a] = piB[(3 * i + a) * V + sm];
      const mat2 U = su2_link(UL, V, i, sm);
      alg_comp(mat_mul(mat_mul(mat_dag(U), alg_mat(xm)), U), xt);
      for (int a = 0; a < 3; ++a) divB[a] += (piB[(3 * i + a) * V + s] - xt[a]) / m->dx;
    }
    const double rhoA = 2.0 * m->e / m->wf2 * vdot(p, q).im;
    out[0] += (divA - rhoA) * (divA - rhoA);
    out[1] += divA * divA;
    out[2] += rhoA * rhoA;
    out[6] += rhoA;
    for (int a = 1; a <= 3; ++a) {
      const double rhoB = m->g / m->wf2 * vdot(p, mat_vec(pauli(a), q)).im;
      out[3] += (divB[a - 1] - rhoB) * (divB[a - 1] - rhoB);
      out[4] += divB[a - 1] * divB[a - 1];
      out[5] += rhoB * rhoB;
      out[6 + a] += rhoB;
    }
  }
}

/* Observables; e[0..8] as su2_energies, e[9] = b, e[10] = Hubble-constraint residual,
   e[11] = Gauss residual of U(1), e[12] = of SU(2), e[13..16] = <components of Phi>,
   e[17] = <|Phi|^2>.  Staggered (lf = 1): kinetic semi-sums, b_n the mean of the two
   half-step values, as orc_u1_lf_observe. */
static void su2_observe(const orc_su2* m, const double* phi, const double* pi, const double* VL, const double* UL,
                        const double* piA, const double* piB, double a, double b, double h, int lf, double* e) {
  const int64_t V = (int64_t)m->N * m->N * m->N;
  double s[ORC_SU2_NS];
  double bn = b;
  if (lf) {
    double* Kp = (double*)malloc(sizeof(double) * 4 * V);
    double* KA = (double*)malloc(sizeof(double) * 3 * V);
    double* KB = (double*)malloc(sizeof(double) * 9 * V);
    orc_su2_kernels(m, a, phi, VL, UL, Kp, KA, KB);
    double kp1 = 0.0, ka1 = 0.0, kb1 = 0.0;
    for (int64_t i = 0; i < 4 * V; ++i) { const double v = pi[i] + h * Kp[i]; kp1 += v * v; }
    for (int64_t i = 0; i < 3 * V; ++i) { const double v = piA[i] + h * KA[i]; ka1 += v * v; }
    for (int64_t i = 0; i < 9 * V; ++i) { const double v = piB[i] + h * KB[i]; kb1 += v * v; }
    const double kp0 = sum_sq(pi, 4 * V), ka0 = sum_sq(piA, 3 * V), kb0 = sum_sq(piB, 9 * V);
    orc_su2_sums(m, phi, NULL, VL, UL, NULL, NULL, s);
    su2_energies(m, a, s, 0.5 * (kp0 + kp1) / (double)V, 0.5 * (ka0 + ka1) / (double)V,
                 0.5 * (kb0 + kb1) / (double)V, e);
    if (m->expand) bn = 0.5 * (b + b + h * orc_su2_Ka(m, a, e));
    free(Kp);
    free(KA);
    free(KB);
  } else {
    orc_su2_sums(m, phi, pi, VL, UL, piA, piB, s);
    su2_energies(m, a, s, -1.0, -1.0, -1.0, e);
  }
  double hc = 0.0;
  if (m->expand) {
    const double rho = e[0] + e[1] + e[2] + e[3] + e[4] + e[5] + e[6];
    const double rhs = m->fmp2 / 3.0 * pow(a, 2.0 * (m->alpha + 1.0)) * rho;
    hc = fabs(bn * bn - rhs) / (bn * bn);
  }
  double g[10];
  orc_su2_gauss(m, phi, pi, UL, piA, piB, g);
  e[9] = bn;
  e[10] = hc;
  e[11] = sqrt(g[0]) / (sqrt(g[1]) + sqrt(g[2]));
  e[12] = sqrt(g[3]) / (sqrt(g[4]) + sqrt(g[5]));
  for (int k = 0; k < 4; ++k) e[13 + k] = s[8 + k];
  e[17] = s[12];
}

void orc_su2_lf_observe(const orc_su2* m, const double* phi, const double* pi, const double* VL, const double* UL,
                        const double* piA, const double* piB, double a, double b, double h, double* e) {
  su2_observe(m, phi, pi, VL, UL, piA, piB, a, b, h, 1, e);
}

void orc_su2_sync_observe(const orc_su2* m, const double* phi, const double* pi, const double* VL,
                          const double* UL, const double* piA, const double* piB, double a, double b, double* e) {
  su2_observe(m, phi, pi, VL, UL, piA, piB, a, b, 0.0, 0, e);
}
