/*
 * Drives every entry point of the C oracle on tiny lattices, for a build
 * under AddressSanitizer and UndefinedBehaviorSanitizer: each buffer is
 * allocated at exactly the size its entry point documents, so a read or
 * write one element past it, a use of freed memory, a leak or an undefined
 * integer operation ends the run with a report.  Every result is also checked
 * to be finite.
 *
 * The oracle source is compiled into this program (one translation unit), so
 * its model structures and internal sizes are the oracle's own.  Inputs are a
 * smooth seeded state near the models' homogeneous values (an LCG, nothing of
 * the method's arithmetic).
 *
 * PLANT (a compile-time switch, 0 by default) builds a variant with one
 * deliberate mistake, so that a test can show each sanitizer reports it:
 * 1 gives the oracle a field array one element short, 2 leaks a buffer,
 * 3 overflows a signed integer.
 */
#include <limits.h>
#include <stdio.h>

#ifndef PLANT
#define PLANT 0
#endif

#include "../../oracle/oracle.c"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static double urand(void) {   /* uniform in [-0.5, 0.5) */
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

static double* alloc(int64_t n) {
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
  return p;
}

static void fill(double* p, int64_t n, double base, double amp) {
  for (int64_t i = 0; i < n; ++i) p[i] = base + amp * urand();
}

static int failures = 0;

static void finite(const char* what, const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(p[i])) {
      fprintf(stderr, "%s[%lld] = %g is not finite\n", what, (long long)i, p[i]);
      ++failures;
      return;
    }
}

/* unit links with small random angles: (re, im) pairs, or angles for the
   non-compact form */
static void unit_links(double* L, int64_t V, int ndir, int noncompact) {
  for (int i = 0; i < ndir; ++i)
    for (int64_t s = 0; s < V; ++s) {
      const double th = 0.2 * urand();
      if (noncompact) {
        L[i * V + s] = th;
      } else {
        L[(2 * i) * V + s] = cos(th);
        L[(2 * i + 1) * V + s] = sin(th);
      }
    }
}

/* unit quaternions near the identity, (3 directions, 4 components, V) */
static void unit_quats(double* U, int64_t V) {
  for (int i = 0; i < 3; ++i)
    for (int64_t s = 0; s < V; ++s) {
      double q[4] = {1.0, 0.1 * urand(), 0.1 * urand(), 0.1 * urand()};
      const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      for (int c = 0; c < 4; ++c) U[(4 * i + c) * V + s] = q[c] / n;
    }
}

static const double TWO_PI = 6.283185307179586476925;

/* Yoshida's fourth-order triple jump, from its closed form */
static double VV4[3];
static void set_vv4(void) {
  const double c = cbrt(2.0);
  VV4[0] = VV4[2] = 1.0 / (2.0 - c);
  VV4[1] = -c / (2.0 - c);
}

static void run_scalar(int N, int nf, int expand) {
  orc_scalar m;
  memset(&m, 0, sizeof m);
  m.N = N; m.nf = nf; m.expand = expand;
  m.dx = TWO_PI / (0.6 * N); m.alpha = 1.0; m.fmp2 = 1e-2;
  m.m2[0] = 0.1; m.m2[1] = 0.05; m.lambda = 1.0; m.q = 100.0;
  const int64_t V = (int64_t)N * N * N, n = nf * V;
  const int64_t nphi = n - (PLANT == 1);
  double *phi = alloc(nphi), *pi = alloc(n), *K = alloc(n);
  double sums[4 * 2 + 3], e[16];
  fill(phi, nphi, 1.0, 0.02);
  fill(pi, n, 0.0, 0.02);
  double a = 1.0, b = expand ? 0.1 : 0.0;
  orc_scalar_kernel(&m, a, phi, K);
  finite("scalar K", K, n);
  orc_scalar_sums(&m, phi, pi, sums);
  finite("scalar sums", sums, 4 * nf + 3);
  orc_scalar_energies(&m, a, sums, e);
  double ka = orc_Ka(&m, a, e[0], e[1], e[2]), hc = orc_hc_rhs(&m, a, 1.0);
  finite("scalar Ka", &ka, 1);
  finite("scalar hc", &hc, 1);

  orc_lf_startup(&m, phi, pi, &a, &b, 0.01);
  orc_lf_steps(&m, phi, pi, &a, &b, 0.01, 3);
  orc_lf_observe(&m, phi, pi, a, b, 0.01, e);
  finite("scalar lf phi", phi, n);
  finite("scalar lf e", e, 16);

  const double vv2 = 1.0;
  orc_vv_steps(&m, phi, pi, &a, &b, 0.01, &vv2, 1, 2);
  orc_vv_steps(&m, phi, pi, &a, &b, 0.01, VV4, 3, 2);
  orc_sync_observe(&m, phi, pi, a, b, e);
  finite("scalar vv pi", pi, n);
  finite("scalar vv e", e, 16);
  free(phi); free(pi);
  if (PLANT != 2) free(K);
}

static void run_u1(int N, int noncompact, int expand) {
  orc_u1 m;
  memset(&m, 0, sizeof m);
  m.N = N; m.expand = expand; m.noncompact = noncompact;
  m.dx = TWO_PI / (0.6 * N); m.alpha = 1.0; m.fmp2 = 1e-2;
  m.lambda = 1.0; m.m2 = 0.1; m.e = 0.5; m.wf2 = 1e-4;
  const int64_t V = (int64_t)N * N * N, nl = (noncompact ? 3 : 6) * V;
  double *phi = alloc(2 * V), *pi = alloc(2 * V), *L = alloc(nl), *piA = alloc(3 * V);
  double *Kp = alloc(2 * V), *KA = alloc(3 * V);
  double sums[9], e[13], g[4];
  fill(phi, 2 * V, 0.5, 0.05);
  fill(pi, 2 * V, 0.0, 0.05);
  unit_links(L, V, 3, noncompact);
  fill(piA, 3 * V, 0.0, 0.02);
  double a = 1.0, b = expand ? 0.1 : 0.0;
  orc_u1_kernels(&m, a, phi, L, Kp, KA);
  finite("u1 Kphi", Kp, 2 * V);
  finite("u1 KA", KA, 3 * V);
  orc_u1_sums(&m, phi, pi, L, piA, sums);
  finite("u1 sums", sums, 9);

  orc_u1_lf_startup(&m, phi, pi, L, piA, &a, &b, 0.01);
  orc_u1_lf_steps(&m, phi, pi, L, piA, &a, &b, 0.01, 3);
  orc_u1_lf_observe(&m, phi, pi, L, piA, a, b, 0.01, e);
  finite("u1 lf e", e, 13);

  const double vv2 = 1.0;
  orc_u1_vv_steps(&m, phi, pi, L, piA, &a, &b, 0.01, &vv2, 1, 2);
  orc_u1_vv_steps(&m, phi, pi, L, piA, &a, &b, 0.01, VV4, 3, 1);
  orc_u1_sync_observe(&m, phi, pi, L, piA, a, b, e);
  finite("u1 vv e", e, 13);
  double ka = orc_u1_Ka(&m, a, e);
  finite("u1 Ka", &ka, 1);
  orc_u1_gauss(&m, phi, pi, piA, g);
  finite("u1 gauss", g, 4);
  finite("u1 links", L, nl);
  free(phi); free(pi); free(L); free(piA); free(Kp); free(KA);
}

static void run_su2(int N, int expand) {
  orc_su2 m;
  memset(&m, 0, sizeof m);
  m.N = N; m.expand = expand;
  m.dx = TWO_PI / (0.6 * N); m.alpha = 1.0; m.fmp2 = 1e-2;
  m.lambda = 1.0; m.m2 = 0.1; m.e = 0.1; m.g = 0.2; m.wf2 = 1e-4;
  const int64_t V = (int64_t)N * N * N;
  double *phi = alloc(4 * V), *pi = alloc(4 * V), *VL = alloc(6 * V), *UL = alloc(12 * V);
  double *piA = alloc(3 * V), *piB = alloc(9 * V);
  double *Kp = alloc(4 * V), *KA = alloc(3 * V), *KB = alloc(9 * V);
  double sums[ORC_SU2_NS], e[18], g[10];
  fill(phi, 4 * V, 0.5, 0.05);
  fill(pi, 4 * V, 0.0, 0.05);
  unit_links(VL, V, 3, 0);
  unit_quats(UL, V);
  fill(piA, 3 * V, 0.0, 0.02);
  fill(piB, 9 * V, 0.0, 0.02);
  double a = 1.0, b = expand ? 0.1 : 0.0;
  orc_su2_kernels(&m, a, phi, VL, UL, Kp, KA, KB);
  finite("su2 Kphi", Kp, 4 * V);
  finite("su2 KA", KA, 3 * V);
  finite("su2 KB", KB, 9 * V);
  orc_su2_sums(&m, phi, pi, VL, UL, piA, piB, sums);
  finite("su2 sums", sums, ORC_SU2_NS);

  orc_su2_lf_startup(&m, phi, pi, VL, UL, piA, piB, &a, &b, 0.01);
  orc_su2_lf_steps(&m, phi, pi, VL, UL, piA, piB, &a, &b, 0.01, 3);
  orc_su2_lf_observe(&m, phi, pi, VL, UL, piA, piB, a, b, 0.01, e);
  finite("su2 lf e", e, 18);

  const double vv2 = 1.0;
  orc_su2_vv_steps(&m, phi, pi, VL, UL, piA, piB, &a, &b, 0.01, &vv2, 1, 2);
  orc_su2_vv_steps(&m, phi, pi, VL, UL, piA, piB, &a, &b, 0.01, VV4, 3, 1);
  orc_su2_sync_observe(&m, phi, pi, VL, UL, piA, piB, a, b, e);
  finite("su2 vv e", e, 18);
  double ka = orc_su2_Ka(&m, a, e);
  finite("su2 Ka", &ka, 1);
  orc_su2_gauss(&m, phi, pi, UL, piA, piB, g);
  finite("su2 gauss", g, 10);
  finite("su2 UL", UL, 12 * V);
  free(phi); free(pi); free(VL); free(UL); free(piA); free(piB); free(Kp); free(KA); free(KB);
}

int main(void) {
  set_vv4();
  uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out4[4];
  orc_philox4x32_10(ctr, key, out4);
  uint32_t* stream = (uint32_t*)malloc(sizeof(uint32_t) * 4 * 37);
  orc_philox_stream(7, 1, 2, 37, stream);
  free(stream);
  if (orc_num_threads() < 1) ++failures;
  if (PLANT == 3) {
    volatile int big = INT_MAX;
    const int over = big + 1;
    printf("%d\n", over);
  }

  /* odd and even sides: the periodic wrap at both ends of every axis */
  for (int N = 4; N <= 5; ++N)
    for (int expand = 0; expand <= 1; ++expand) {
      run_scalar(N, 1, expand);
      run_scalar(N, 2, expand);
      run_u1(N, 0, expand);
      run_u1(N, 1, expand);
      run_su2(N, expand);
    }
  if (failures) {
    fprintf(stderr, "%d non-finite results\n", failures);
    return 1;
  }
  printf("oracle driver ok\n");
  return 0;
}
