"""Seeded synthetic workloads and inputs.

This module holds the workload recipes (lattice sizes, couplings, time steps,
seeds) and seeded random lattice states.  It contains none of the method's
arithmetic: no kicks, drifts, energies or spectra.  Both the HIP path and the
test oracle read their inputs from here.

Units are the paper's program variables (Sec. 4.1): fields in units of f_*,
times and lengths in units of 1/omega_*, alpha-time with alpha = 1.
"""
from __future__ import annotations

import math

import numpy as np

# f_*/m_p for the monomial p = 4 model with M = 10 m_p: f_* = phi_* =
# (M/2) arcsinh(sqrt(2) p m_p / M) (Sec. 8.1, slow-roll end).
FSTAR_OVER_MP = 5.0 * math.asinh(math.sqrt(2.0) * 4.0 / 10.0)


def config1() -> dict:
    """Single real scalar, lambda phi^4/4 with lambda = 1e-4, 32^3, kIR = 0.1,
    FP64, staggered leapfrog, dt = 0.01, 1000 steps, phi0 = 1, vacuum
    fluctuations with (w*/f*) = 1, self-consistent expansion."""
    return dict(name="scalar1_32_lf2_fp64", model="scalar", nf=1, N=32, kIR=0.1, dt=0.01,
                nsteps=1000, alpha=1.0, fstar_over_mp=FSTAR_OVER_MP, omega_over_f=1.0,
                m2=(0.0, 0.0), lam=1e-4, q=0.0, phi0=(1.0, 0.0), dphi0=(0.0, 0.0),
                integrator="lf2", precision="fp64", expansion=True, ic="vacuum", seed=1, a0=1.0)


def config2(q: float = 100.0, integrator: str = "vv2", N: int = 256, seed: int | None = None) -> dict:
    """Two scalars, V = phi^4/4 + q phi^2 chi^2/2 (program units, p = 4),
    256^3, kIR = 0.6, FP32 state with FP64 sums, VV2 or VV4, dt = 0.005,
    vacuum fluctuations with (w*/f*)^2 = lambda = 1e-4."""
    if seed is None:
        seed = 2 if q == 100.0 else 3
    return dict(name=f"scalar2_{N}_{integrator}_q{q:g}_fp32", model="scalar", nf=2, N=N, kIR=0.6,
                dt=0.005, nsteps=20000, alpha=1.0, fstar_over_mp=FSTAR_OVER_MP, omega_over_f=1e-2,
                m2=(0.0, 0.0), lam=1.0, q=float(q), phi0=(1.0, 0.0), dphi0=(0.0, 0.0),
                integrator=integrator, precision="fp32", expansion=True, ic="vacuum", seed=seed,
                a0=1.0)


def config3(N: int = 192) -> dict:
    """Abelian-Higgs with compact U(1) links: e = 0.5, lambda = 1, 192^3,
    kIR = 0.6, FP32, staggered leapfrog dt = 0.01, 1000 steps, Gauss check
    every 100 steps."""
    s = 1.0 / math.sqrt(2.0)
    return dict(name=f"u1higgs_{N}_lf2_fp32", model="u1", nf=2, N=N, kIR=0.6, dt=0.01, nsteps=1000,
                alpha=1.0, fstar_over_mp=FSTAR_OVER_MP, omega_over_f=1e-2, m2=(0.0, 0.0), lam=1.0,
                q=0.0, e=0.5, phi0=(s, s), dphi0=(0.0, 0.0), integrator="lf2", precision="fp32",
                expansion=True, ic="vacuum", seed=5, a0=1.0)


def config3_noncompact(N: int = 192) -> dict:
    """The same Abelian-Higgs physics with the non-compact gauge field of
    Sec. 5.2 (A_i evolved directly, quadratic magnetic energy)."""
    c = config3(N)
    c["model"] = "u1nc"
    c["name"] = f"u1nc_higgs_{N}_lf2_fp32"
    return c


def config_su2u1(N: int = 128, integrator: str = "vv2") -> dict:
    """Doublet with SU(2) x U(1) links, the paper's p = 4 working example
    without its singlet: V = |Phi|^4 (program units), resonance parameters
    q_A = e^2/lambda and q_B = g^2/(4 lambda) both 100 with lambda = (w*/f*)^2 =
    1e-4, so e = 0.1 and g = 0.2; 128^3, kIR = 0.6, dt = 0.01, every real
    component of Phi starting at 1/2 (|Phi| = 1/sqrt 2), FP32, seed 6."""
    return dict(name=f"su2u1_{N}_{integrator}_fp32", model="su2u1", nf=4, N=N, kIR=0.6, dt=0.01, nsteps=1000,
                alpha=1.0, fstar_over_mp=FSTAR_OVER_MP, omega_over_f=1e-2, m2=(0.0, 0.0), lam=1.0, q=0.0,
                e=0.1, g=0.2, phi0=(0.5, 0.5, 0.5, 0.5), dphi0=(0.0, 0.0, 0.0, 0.0), integrator=integrator,
                precision="fp32", expansion=True, ic="vacuum", seed=6, a0=1.0)


def config4_runs(nruns: int = 96, sizes=(32, 64, 96), nsteps: int = 5000) -> list:
    """96 independent two-scalar VV2 runs, sizes split evenly among 32^3,
    64^3, 96^3, q = 10^(1+3u) with u uniform from a seeded generator, seeds
    4000 + i."""
    rng = np.random.default_rng(4000)
    u = rng.random(nruns)
    runs = []
    for i in range(nruns):
        N = sizes[i * len(sizes) // nruns]
        c = config2(q=float(10.0 ** (1.0 + 3.0 * u[i])), integrator="vv2", N=N, seed=4000 + i)
        c["nsteps"] = nsteps
        c["name"] = f"batch_{i}_{N}"
        runs.append(c)
    return runs


def small(cfg: dict, N: int) -> dict:
    """The same physics on an N^3 lattice (kIR kept, so the box shrinks)."""
    c = dict(cfg)
    c["N"] = N
    c["name"] = cfg["name"] + f"_N{N}"
    return c


def random_state(cfg: dict, seed: int, amp: float = 0.1, mom: float = 0.1) -> dict:
    """A seeded random smooth-ish lattice state for kernel parity tests:
    homogeneous values plus uniform noise of amplitude amp (fields) and mom
    (momenta).  Shapes (nf, N, N, N), FP64."""
    rng = np.random.default_rng(seed)
    N, nf = int(cfg["N"]), int(cfg["nf"])
    phi0 = list(cfg.get("phi0", (1.0, 0.0)))
    phi = np.empty((nf, N, N, N))
    pi = np.empty((nf, N, N, N))
    for f in range(nf):
        phi[f] = phi0[f] + amp * (rng.random((N, N, N)) - 0.5)
        pi[f] = mom * (rng.random((N, N, N)) - 0.5)
    return {"phi": phi, "pi": pi}


def random_u1_state(N: int, seed: int, amp: float = 0.1, link_angle: float = 0.2,
                    emom: float = 0.05) -> dict:
    """Seeded random compact-U(1) lattice state: complex scalar (re, im)
    around (1/2, 1/2), momenta, unit links with random angles, link momenta.
    Shapes: phi, pi (2, N, N, N); links (3, 2, N, N, N) as (re, im);
    piA (3, N, N, N).  FP64."""
    rng = np.random.default_rng(seed)
    phi = 0.5 + amp * (rng.random((2, N, N, N)) - 0.5)
    pi = amp * (rng.random((2, N, N, N)) - 0.5)
    th = link_angle * (rng.random((3, N, N, N)) - 0.5)
    links = np.stack([np.cos(th), np.sin(th)], axis=1)
    piA = emom * (rng.random((3, N, N, N)) - 0.5)
    return {"phi": phi, "pi": pi, "links": links, "piA": piA}


def mlp_init(seed: int, widths=(24, 256, 256, 256, 64), bias_scale: float = 0.0) -> dict:
    """Glorot-uniform weights W_l (out, in) and biases uniform in
    [-bias_scale, bias_scale] for the spectrum surrogate, from a seeded
    generator."""
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(len(widths) - 1):
        fi, fo = widths[l], widths[l + 1]
        lim = math.sqrt(6.0 / (fi + fo))
        p[f"W{l + 1}"] = rng.uniform(-lim, lim, (fo, fi))
        p[f"b{l + 1}"] = rng.uniform(-bias_scale, bias_scale, fo) if bias_scale else np.zeros(fo)
    return p


def config5_train_runs(nruns: int = 2000, N: int = 64, nsteps: int = 5000, seed0: int = 10000) -> list:
    """Training runs of the spectrum surrogate: the two-field model of
    config2 on N^3, VV2, q = 10^(1+3u) with u uniform from a generator seeded
    with seed0, lattice seeds seed0 + i."""
    rng = np.random.default_rng(seed0)
    u = rng.random(nruns)
    runs = []
    for i in range(nruns):
        c = config2(q=float(10.0 ** (1.0 + 3.0 * u[i])), integrator="vv2", N=N, seed=seed0 + i)
        c["nsteps"] = nsteps
        c["name"] = f"surr_train_{i}"
        runs.append(c)
    return runs


def config5_heldout_runs(nq: int = 64, nseeds: int = 8, N: int = 64, nsteps: int = 5000,
                         seed0: int = 20000) -> list:
    """Held-out scoring runs: nq new q values (log-uniform in [10, 1e4] from a
    generator seeded with seed0), nseeds lattice realisations each, seeds
    seed0 + nseeds * iq + s.  Returned grouped by q."""
    rng = np.random.default_rng(seed0)
    qs = 10.0 ** (1.0 + 3.0 * rng.random(nq))
    runs = []
    for iq in range(nq):
        for s in range(nseeds):
            c = config2(q=float(qs[iq]), integrator="vv2", N=N, seed=seed0 + nseeds * iq + s)
            c["nsteps"] = nsteps
            c["name"] = f"surr_heldout_{iq}_{s}"
            runs.append(c)
    return runs
