/*
 * cosmolat.h -- C ABI of the MI355X (gfx950) lattice library.
 *
 * The library advances interacting scalar fields (and a compact U(1) gauge
 * field) on a periodic N^3 lattice in a self-consistently expanding FLRW
 * background, following Figueroa, Florio, Torrenti, Valkenburg, "The art of
 * simulating the early Universe - Part I" (arXiv:2006.15122).  All variables
 * are the paper's program variables (Sec. 4.1): fields in units of f_*,
 * times and lengths in units of 1/omega_*, alpha-time d eta = a^-alpha w_* dt.
 *
 * Conventions shared by every entry point
 *  - Return value 0 on success, a negative LAT_E* code on failure; the text
 *    of the last failure of the calling thread is lattice_last_error().
 *  - Memory crossing the boundary is owned by the caller.  Device memory
 *    (the workspace) is allocated by the caller; the library never calls
 *    hipMalloc.  Host arrays are only read or written during the call.
 *  - Device work is issued on the HIP stream given to lattice_init.  Calls
 *    that return host data synchronise that stream; lattice_step does not.
 *  - One handle per host thread; handles are independent.
 *  - Site (x, y, z), 0 <= x, y, z < N, has linear index (x*N + y)*N + z
 *    (z fastest).  Host arrays are FP64, component-major: component c of a
 *    multi-component array starts at c*N^3.
 */
#ifndef COSMOLAT_H
#define COSMOLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes */
#define LAT_OK 0
#define LAT_EINVAL (-1)     /* bad parameters, unsupported N, Courant bound  */
#define LAT_ENOMEM (-2)     /* workspace or caller buffer too small          */
#define LAT_EHIP (-3)       /* HIP runtime failure (text in last_error)      */
#define LAT_ENONFINITE (-4) /* NaN or Inf in the volume averages             */
#define LAT_ESTATE (-5)     /* call out of order, or invalid state           */

/* Models */
#define LAT_MODEL_SCALAR 0  /* nf = 1 or 2 real scalars (Sec. 4):
                               V = sum_f m2[f] phi_f^2/2 + lambda phi_0^4/4
                                   + q phi_0^2 phi_1^2/2                      */
#define LAT_MODEL_U1 1      /* complex scalar with compact U(1) links (Sec. 5.3):
                               V = lambda |phi|^4 + m2[0] |phi|^2            */
#define LAT_MODEL_U1_NC 2   /* the same with the non-compact gauge field A_i
                               (Sec. 5.2): A' = a^{-(1-alpha)} pi_A, magnetic
                               kernel sum_j (D-_j D+_j A_i - D-_j D+_i A_j),
                               E_G^A from F_ij = D+_i A_j - D+_j A_i         */
#define LAT_MODEL_SU2U1 3   /* doublet Phi = (phi_0 + i phi_1, phi_2 + i phi_3)
                               / sqrt 2 with compact SU(2) and U(1) links
                               (Sec. 6): V = lambda |Phi|^4 + m2[0] |Phi|^2,
                               U(1) coupling e, SU(2) coupling g; nf = 4.
                               Every real component starts at phi0[0] (and
                               dphi0[0]), the equal amplitudes of Sec. 7.2 */

/* Integrators (Sec. 3.3-3.4, 4.2-4.3) */
#define LAT_LF2 0   /* staggered leapfrog, scheme III (pi = a^{3-alpha} phi')    */
#define LAT_VV2 1   /* velocity Verlet                                          */
#define LAT_VV4 2   /* Yoshida composition of VV2, 3 sub-steps                  */
#define LAT_VV6 3   /* Yoshida, 7 sub-steps (appendix table of coefficients)     */
#define LAT_VV8 4   /* Yoshida, 15 sub-steps                                     */
#define LAT_VV10 5  /* Yoshida, 31 sub-steps                                     */

/* Storage precision of fields and momenta.  Volume averages, a and b are
   always accumulated and kept in FP64. */
#define LAT_FP64 0
#define LAT_FP32 1

/* Initial conditions */
#define LAT_IC_VACUUM 0       /* homogeneous values + vacuum fluctuations (Sec. 7) */
#define LAT_IC_HOMOGENEOUS 1  /* homogeneous values only                           */

typedef struct lattice_params {
  int32_t model;       /* LAT_MODEL_*                                      */
  int32_t nf;          /* LAT_MODEL_SCALAR: 1 or 2; LAT_MODEL_U1(_NC): 2    */
  int32_t N;           /* sites per side: multiple of 32, 32 <= N <= 1024  */
  int32_t integrator;  /* LAT_LF2, LAT_VV2, LAT_VV4                         */
  int32_t precision;   /* LAT_FP64 or LAT_FP32                              */
  int32_t expansion;   /* 1: self-consistent a(eta); 0: flat, a = 1, b = 0  */
  int32_t ic;          /* LAT_IC_*                                          */
  int32_t reserved;
  uint64_t seed;       /* random seed of the initial fluctuations           */
  double kIR;          /* infrared momentum 2 pi/(N dx)                     */
  double dt;           /* time step (program units)                         */
  double alpha;        /* alpha-time exponent                               */
  double fstar_over_mp;/* f_* / m_p                                         */
  double omega_over_f; /* w_* / f_*, amplitude factor of the vacuum spectrum */
  double m2[2];        /* mass terms                                         */
  double lambda;       /* quartic coupling                                   */
  double q;            /* phi^2 chi^2 coupling                               */
  double e;            /* gauge coupling g_A Q_A (LAT_MODEL_U1, U1_NC)       */
  double phi0[2];      /* homogeneous field values                           */
  double dphi0[2];     /* homogeneous d phi / d eta                          */
  double a0;           /* initial scale factor (1)                           */
  double kcut;         /* 0: no cut; else fluctuations only for k <= kcut    */
  double g;            /* SU(2) gauge coupling g_B Q_B (LAT_MODEL_SU2U1)     */
} lattice_params;

/* Homogeneous variables of a state.  For LAT_LF2, staggered = 1 means the
   momenta and b are half a step behind phi and a (pi_{n-1/2}, b_{n-1/2}). */
typedef struct lattice_scalars {
  double a;
  double b;            /* a' = d a / d eta                                  */
  double eta;
  int64_t step;
  int32_t staggered;
  int32_t reserved;
} lattice_scalars;

/* Observables (Sec. 4.4, 5.4), all FP64 volume averages in program units. */
typedef struct lattice_obs {
  double eta, a, b;    /* b at the same time as a (LF2: mean of the two    */
                       /* neighbouring half-step values)                   */
  double H;            /* b / a                                             */
  double EK, EG, EV;   /* total kinetic, gradient, potential energy         */
  double EV_term[3];   /* mass, quartic, interaction parts of EV            */
  double EK_f[2];      /* kinetic energy per scalar field                   */
  double EG_f[2];      /* gradient energy per scalar field                  */
  double mean_f[2];    /* <phi_f> (U1: <Re phi>, <Im phi>)                  */
  double meansq_f[2];  /* <phi_f^2>                                         */
  double EK_A, EG_A;   /* U(1) electric and magnetic energy                 */
  double rho, p, w;    /* energy density, pressure, p/rho                   */
  double hc;           /* Hubble-constraint residual |b^2 - rhs| / b^2      */
  double gauss;        /* U(1) Gauss-law residual (NaN for scalars)         */
  int64_t step;
  int32_t staggered;
  int32_t reserved;
  double EK_B, EG_B;   /* SU(2) electric and magnetic energy (Sec. 6.3.1)   */
  double gauss_B;      /* SU(2) Gauss-law residual                          */
  double mean_lo[2];   /* SU(2) x U(1): <Re Phi_1>, <Im Phi_1>; mean_f holds */
                       /* <Re Phi_0>, <Im Phi_0> and meansq_f[0] <|Phi|^2>  */
} lattice_obs;

typedef struct lattice lattice_t;

/* Device bytes lattice_init needs for p.  Errors: LAT_EINVAL. */
int lattice_workspace_size(const lattice_params* p, size_t* bytes);

/* Validate p, carve dev_ws (device memory of ws_bytes >= the size above,
   owned by the caller and kept alive until lattice_destroy), and build the
   initial state on the device: homogeneous values plus, for LAT_IC_VACUUM,
   the vacuum fluctuations of Sec. 7.1 (Rayleigh moduli and uniform phases
   drawn from Philox4x32-10 keyed by seed), b fixed by the Hubble constraint.
   hip_stream is a hipStream_t (NULL: the default stream).
   Errors: LAT_EINVAL (parameters, Courant bound dt <= dx/sqrt(3)),
   LAT_ENOMEM (ws_bytes too small), LAT_EHIP. */
int lattice_init(const lattice_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                 lattice_t** out);

/* Replace the state by host FP64 arrays (converted to the storage
   precision).  Scalar model: fields and momenta are nf*N^3 values.  U1:
   fields and momenta are 2*N^3 (Re, Im of the complex scalar phi), links
   3*2*N^3 (direction i, then Re/Im, of V_i), link_momenta 3*N^3 (pi_A,i).
   U1_NC: as U1 but links holds the gauge field A_i, 3*N^3 values (the
   link is V_i = exp(-i e dx A_i)).  links and link_momenta must be NULL for
   scalar models.
   Errors: LAT_EINVAL (NULL arrays), LAT_ENONFINITE, LAT_EHIP. */
int lattice_set_state(lattice_t* h, const double* fields, const double* momenta,
                      const double* links, const double* link_momenta,
                      const lattice_scalars* s);

/* Copy the state to host FP64 arrays of the sizes above (any may be NULL to
   skip it).  Synchronises the stream.  Errors: LAT_EHIP. */
int lattice_get_state(lattice_t* h, double* fields, double* momenta, double* links,
                      double* link_momenta, lattice_scalars* s);

/* Advance nsteps >= 0 full time steps with the configured integrator:
   VV2/VV4 end synchronised at an integer time; LF2 ends staggered
   (phi_n, a_n; pi_{n-1/2}, b_{n-1/2}).  Asynchronous on the stream.
   Errors: LAT_EINVAL (nsteps < 0), LAT_EHIP. */
int lattice_step(lattice_t* h, int64_t nsteps);

/* Observables of the current state.  Synchronises the stream.
   Errors: LAT_ENONFINITE (NaN/Inf in a volume average), LAT_EHIP. */
int lattice_energies(lattice_t* h, lattice_obs* out);

/* Spectrum selectors of the U(1) models that add components shell by shell
   (Sec. 5.4.2): the complex scalar |Re phi(n~)|^2 + |Im phi(n~)|^2, the same
   for its momentum, the electric field sum_i |E_i(n~)|^2 with
   E_i = pi_A,i / a^{1-alpha} (a of the current state; in a staggered state
   pi_A is the stored half-step value), and the magnetic field
   sum_i |B_i(n~)|^2 with B_i = Im V_jk / (e dx^2) for (i, j, k) cyclic
   (compact links; the factor i printed before Im is read as a typo) or
   B_i = D+_j A_k - D+_k A_j (non-compact).  B is computed in FP64 from the
   stored links and transformed in the storage precision. */
#define LAT_SPEC_U1_PHI 32
#define LAT_SPEC_U1_PI 33
#define LAT_SPEC_U1_E 34
#define LAT_SPEC_U1_B 35

/* lattice_energies for callers that cannot allocate device memory or hold a
   workspace for it (code under HIP graph capture, tight serving loops,
   harnesses that forbid allocation): the same passes and kernels, with their
   per-block FP64 partial sums in a 4 MiB static device array of the library
   (one per device, held until the process ends) instead of the workspace
   (SU(2) x U(1) folds those records into 64 in the workspace's second record
   buffer, as lattice_energies does); results are bitwise those of
   lattice_energies.  Allocates nothing.  Calls
   that overlap on one GPU share that array and race; the caller serialises
   them.  Errors: LAT_ENOMEM when the partial sums need more than 4 MiB
   (U(1) lattices above 320^3, SU(2) x U(1) above 192^3, two scalar fields
   above 544^3), and those of lattice_energies. */
int lattice_energies_noalloc(lattice_t* h, lattice_obs* out);

/* Radially binned power spectrum of one field component (Sec. 3.1, eq. of
   the discrete spectrum; Sec. 4.4.2, 5.4.2).  Shell b holds the modes with
   floor(|n~|) = b, b = 0 .. floor(sqrt(3) N / 2).  Per shell: k[b] = mean
   k_IR |n~|, sum_sq[b] = sum |f(n~)|^2 with f(n~) = sum_n e^{+2 pi i n~.n/N}
   f(n), counts[b], and delta[b] = (k_IR b)^3/(2 pi^2) (dx/N)^3 sum_sq[b] /
   (4 pi b^2) for b >= 1 (0 for b = 0).  which: for scalar models 0..nf-1 =
   field f, 16+f = momentum f; for U(1) models 0, 1 = Re, Im phi, 16, 17 =
   Re, Im pi, and the summed LAT_SPEC_U1_* selectors above; for the SU(2) x
   U(1) model 0..3 and 16..19 = the real components of Phi and pi, and
   LAT_SPEC_U1_PHI / LAT_SPEC_U1_PI = their sums.  The stored values are
   transformed in FP64 for either storage precision, and the shell sums are
   FP64; within a block they are added in no fixed order, so results are
   reproducible to FP64 rounding.  Caller-owned host arrays of
   nbins_cap entries; *nbins receives the number of shells.  Synchronises the
   stream.  Errors: LAT_EINVAL (which), LAT_ENOMEM (nbins_cap too small),
   LAT_EHIP. */
int lattice_spectrum(lattice_t* h, int which, int nbins_cap, double* k, double* delta,
                     double* sum_sq, int64_t* counts, int* nbins);

/* The same spectrum reduced on the device to nk values, for training sets
   built without host round trips: log10 of the mode-averaged spectrum
   kbar_b^3/(2 pi^2) (dx/N)^3 sum_sq[b] / counts[b] (Sec. 3.1 with the
   average over the modes of each shell) at nk wavenumbers
   k_j = k_IR (b_max)^(j/(nk-1)), b_max = floor(sqrt(3) N / 2), linear in
   log10 k between the centres (mean k) of the shells b >= 1 that hold modes
   and positive power, constant beyond the first and last such shell
   (-inf if there is none).  dev_out: caller-owned device array of nk FP32.
   Asynchronous on the stream.  Errors: LAT_EINVAL (which, nk outside
   [2, 4096], NULL), LAT_EHIP. */
int lattice_spectrum_logk(lattice_t* h, int which, int nk, float* dev_out);

/* Release the handle (not the workspace).  Synchronises the stream. */
int lattice_destroy(lattice_t* h);

/* Text of the calling thread's last error ("" if none). */
const char* lattice_last_error(void);

/* Tile shape of the fused pass: threads along z, rows of threads along y,
   rows per thread, x-planes per block.  Scalar lattices compile (64,4,2)
   (64,8,2) (32,8,2) (128,8,2) (256,4,2) (128,4,2) for FP32 two fields, plus
   the full-row tiles (128,16,1) (256,8,1) (512,4,1), valid only where the first
   number equals N: a block holds whole z-rows, four sites per thread, and
   each site's update is bit for bit the general tiles'.  FP64 two fields
   compile (64,4,2) (32,8,2) (32,4,4) and the full-row tiles (128,8,1)
   (256,4,1) (512,2,1) (two sites per thread); other scalar storage and field
   counts (64,4,2) (32,8,2) (32,4,4); U(1) lattices (64,4,2) and
   (32,8,1) in FP32, (32,8,1) in FP64.  lattice_init picks one (the built-in
   autotuner times them for N >= 128, once per model, size, precision,
   integrator and expansion in a process, so that later lattices of the same
   configuration share the tile and with it the order of their FP64 sums);
   this call reports it.  SU(2) x U(1) passes are untiled (0, 0, 0, 0).  */
int lattice_get_tiling(lattice_t* h, int32_t* tz, int32_t* by, int32_t* ry, int32_t* xc);

/* Force a tile shape (for the autotuner and tests).  Errors: LAT_EINVAL if
   the shape is not compiled, does not divide N, or is a full-row tile of
   another N. */
int lattice_set_tiling(lattice_t* h, int32_t tz, int32_t by, int32_t ry, int32_t xc);

/* Kernel timing of the fused pass (scalar or U(1)).  After lattice_pass_timer(h, n),
   the next n stepping-pass launches of lattice_step carry the device's own
   start and stop timestamps of their dispatch (the launch is otherwise the
   same; no work is added or skipped).  lattice_pass_timer_read synchronises
   the stream and returns the summed kernel time of the recorded launches
   and their number, then starts a new count with the same events.
   n = 0 releases the events.
   Errors: LAT_EINVAL, LAT_EHIP. */
int lattice_pass_timer(lattice_t* h, int32_t max_launches);
int lattice_pass_timer_read(lattice_t* h, double* total_ms, int64_t* launches);

/* Device pointer to component c of the current fields (storage precision),
   and the storage element size in bytes; for zero-copy consumers. */
int lattice_field_device_ptr(lattice_t* h, int c, void** ptr, int32_t* elem_bytes);

/* ------------------------------------------------------------------------
 * Batched ensembles: nruns independent scalar lattices advanced together,
 * one batched kernel per pass over the tiles of every run plus one FP64
 * finish block per run; a whole lattice_batch_step call is captured in a
 * HIP graph and launched once.  All runs share model (LAT_MODEL_SCALAR), nf,
 * integrator (LAT_VV2 or LAT_VV4), precision and dt; N (multiple of 32),
 * couplings, kIR and seed may differ per run.
 * ------------------------------------------------------------------------ */
typedef struct lattice_batch lattice_batch_t;

/* Device bytes for the batch (ps: array of nruns parameter sets).
   Errors: LAT_EINVAL. */
int lattice_batch_workspace_size(const lattice_params* ps, int nruns, size_t* bytes);

/* Build every run (its initial state as in lattice_init) inside dev_ws and
   pick a tile shape common to all runs with the autotuner.  hip_stream must
   be a created stream (not NULL) for graph capture.  Errors: LAT_EINVAL
   (mismatched shared parameters), LAT_ENOMEM, LAT_EHIP. */
int lattice_batch_init(const lattice_params* ps, int nruns, void* dev_ws, size_t ws_bytes, void* hip_stream,
                       lattice_batch_t** out);

/* Advance every run by nsteps full steps (synchronised at the end).
   Asynchronous on the stream.  Errors: LAT_EINVAL, LAT_EHIP. */
int lattice_batch_step(lattice_batch_t* b, int64_t nsteps);

/* Observables of every run into out[0 .. nruns-1].  Synchronises.
   Errors: LAT_ENONFINITE, LAT_EHIP. */
int lattice_batch_energies(lattice_batch_t* b, lattice_obs* out);

/* Handle of one run, owned by the batch (valid until lattice_batch_destroy):
   use it for lattice_set_state / get_state / energies / spectrum, or with
   lattice_step to advance that run alone with the single-lattice kernels.
   Errors: LAT_EINVAL. */
int lattice_batch_run(lattice_batch_t* b, int run, lattice_t** out);

/* Tile shape shared by the batched pass (see lattice_set_tiling), and graph
   capture on/off (default on).  Errors: LAT_EINVAL. */
int lattice_batch_get_tiling(lattice_batch_t* b, int32_t* tz, int32_t* by, int32_t* ry, int32_t* xc);
int lattice_batch_set_tiling(lattice_batch_t* b, int32_t tz, int32_t by, int32_t ry, int32_t xc);
int lattice_batch_use_graph(lattice_batch_t* b, int on);

/* Release the batch and its run handles (not the workspace). */
int lattice_batch_destroy(lattice_batch_t* b);

#ifdef __cplusplus
}
#endif
#endif /* COSMOLAT_H */
