"""FP64 CPU oracle for the lattice method of arXiv:2006.15122
("The art of simulating the early Universe - Part I").

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never calls it.

The time-stepping loops live in ``oracle.c`` (plain loops, one pass per line of
the paper's schemes); this module wraps them and adds, in numpy, the initial
conditions (Sec. 7.1) and power spectra (Sec. 3.1, Sec. 4.4.2).  numpy's FFT is
used as a library primitive for the discrete Fourier transform.

Parity status per function is stated in the docstrings; every function here is
pinned by at least one test in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = {False: os.path.join(_HERE, "liboracle.so"), True: os.path.join(_HERE, "liboracle_omp.so")}
_LIBS: dict = {}

# Yoshida weights (Appendix, table of VVn coefficients).
# VV4 is Yoshida's symmetric triple jump, w1 = w3 = 1/(2 - 2^(1/3)),
# w2 = -2^(1/3)/(2 - 2^(1/3)).  The table's printed w2 (-1.702414403875838...)
# differs from this closed form at the 8th digit, so that the printed weights
# would sum to 1 - 2e-8, against the requirement sum w_i = 1 stated with the
# method; the closed form is used (the printed w1 agrees to double precision).
_C3 = 2.0 ** (1.0 / 3.0)


def _sym(half, mid):
    return tuple(half) + (mid,) + tuple(reversed(half))


VV_WEIGHTS = {
    "vv2": (1.0,),
    "vv4": (1.0 / (2.0 - _C3), -_C3 / (2.0 - _C3), 1.0 / (2.0 - _C3)),
    "vv6": _sym((0.78451361047755726382, 0.23557321335935813368, -1.1776799841788710069),
                1.3151863206839112189),
    "vv8": _sym((0.74167036435061295345, -0.40910082580003159400, 0.19075471029623837995,
                 -0.57386247111608226666, 0.29906418130365592384, 0.33462491824529818378,
                 0.31529309239676659663), -0.79688793935291635402),
    "vv10": _sym((-0.48159895600253002870, 0.0036303931544595926879, 0.50180317558723140279,
                  0.28298402624506254868, 0.80702967895372223806, -0.026090580538592205447,
                  -0.87286590146318071547, -0.52373568062510581643, 0.44521844299952789252,
                  0.18612289547097907887, 0.23137327866438360633, -0.52191036590418628905,
                  0.74866113714499296793, 0.066736511890604057532, -0.80360324375670830316),
                 0.91249037635867994571),
}


def build(omp: bool = False, force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, FP64, no fast-math)."""
    so = _SO[omp]
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
               _SRC, "-o", so + ".tmp", "-lm"]
        if omp:
            cmd.insert(1, "-fopenmp")
        subprocess.check_call(cmd)
        os.replace(so + ".tmp", so)
    return so


def lib(omp: bool = False):
    if omp not in _LIBS:
        L = ctypes.CDLL(build(omp))
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_Ka.restype = ctypes.c_double
        L.orc_hc_rhs.restype = ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int
        _LIBS[omp] = L
    return _LIBS[omp]


class Scalar(ctypes.Structure):
    """Parameters of the real-scalar model (Sec. 4)."""
    _fields_ = [("N", ctypes.c_int32), ("nf", ctypes.c_int32), ("expand", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("dx", ctypes.c_double), ("alpha", ctypes.c_double),
                ("fmp2", ctypes.c_double), ("m2", ctypes.c_double * 2), ("lam", ctypes.c_double),
                ("q", ctypes.c_double)]


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice_dx(N: int, kIR: float) -> float:
    """Lattice spacing from k_IR = 2 pi / (N dx) (Sec. 3.1)."""
    return 2.0 * math.pi / (kIR * N)


def scalar_model(cfg: dict) -> Scalar:
    m = Scalar()
    m.N = int(cfg["N"])
    m.nf = int(cfg["nf"])
    m.expand = 1 if cfg.get("expansion", True) else 0
    m.dx = lattice_dx(m.N, cfg["kIR"])
    m.alpha = float(cfg.get("alpha", 1.0))
    m.fmp2 = float(cfg.get("fstar_over_mp", 1.0)) ** 2
    m2 = list(cfg.get("m2", (0.0, 0.0))) + [0.0, 0.0]
    m.m2[0], m.m2[1] = float(m2[0]), float(m2[1])
    m.lam = float(cfg.get("lam", 0.0))
    m.q = float(cfg.get("q", 0.0))
    return m


def _f64(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return x


def kernel(m: Scalar, a: float, phi: np.ndarray) -> np.ndarray:
    phi = _f64(phi)
    K = np.empty_like(phi)
    lib().orc_scalar_kernel(ctypes.byref(m), ctypes.c_double(a), _p(phi), _p(K))
    return K


def vv_steps(m: Scalar, phi, pi, a, b, h, integrator="vv2", nsteps=1, omp=False):
    """nsteps velocity-Verlet (VV2) or Yoshida (VV4) steps, in place (Sec. 4.3.2)."""
    w = np.array(VV_WEIGHTS[integrator], dtype=np.float64)
    ca, cb = ctypes.c_double(a), ctypes.c_double(b)
    lib(omp).orc_vv_steps(ctypes.byref(m), _p(phi), _p(pi), ctypes.byref(ca), ctypes.byref(cb),
                          ctypes.c_double(h), _p(w), ctypes.c_int(len(w)), ctypes.c_int64(nsteps))
    return ca.value, cb.value


def lf_startup(m: Scalar, phi, pi, a, b, h):
    """Synchronised -> staggered start-up of scheme III (pi_{-1/2}, b_{-1/2})."""
    ca, cb = ctypes.c_double(a), ctypes.c_double(b)
    lib().orc_lf_startup(ctypes.byref(m), _p(phi), _p(pi), ctypes.byref(ca), ctypes.byref(cb),
                         ctypes.c_double(h))
    return ca.value, cb.value


def lf_steps(m: Scalar, phi, pi, a, b, h, nsteps=1, omp=False):
    """nsteps staggered-leapfrog steps of scheme III (Sec. 4.2.1), in place."""
    ca, cb = ctypes.c_double(a), ctypes.c_double(b)
    lib(omp).orc_lf_steps(ctypes.byref(m), _p(phi), _p(pi), ctypes.byref(ca), ctypes.byref(cb),
                          ctypes.c_double(h), ctypes.c_int64(nsteps))
    return ca.value, cb.value


def _obs_dict(m: Scalar, e: np.ndarray, a: float) -> dict:
    nf = m.nf
    d = {"a": a, "EK": e[0], "EG": e[1], "EV": e[2], "EV_mass": e[3], "EV_quartic": e[4],
         "EV_int": e[5], "b": e[6 + 4 * nf], "hc": e[7 + 4 * nf]}
    for f in range(nf):
        d[f"EK{f}"] = e[6 + 4 * f]
        d[f"EG{f}"] = e[7 + 4 * f]
        d[f"mean{f}"] = e[8 + 4 * f]
        d[f"meansq{f}"] = e[9 + 4 * f]
    rho = e[0] + e[1] + e[2]
    d["rho"] = rho
    d["p"] = e[0] - e[1] / 3.0 - e[2]
    d["w"] = d["p"] / rho if rho != 0 else 0.0
    return d


def sync_observe(m: Scalar, phi, pi, a, b) -> dict:
    """Energies, means and Hubble-constraint residual of a synchronised state."""
    e = np.zeros(16)
    lib().orc_sync_observe(ctypes.byref(m), _p(_f64(phi)), _p(_f64(pi)), ctypes.c_double(a),
                           ctypes.c_double(b), _p(e))
    return _obs_dict(m, e, a)


def lf_observe(m: Scalar, phi, pi, a, b, h) -> dict:
    """Observables of a staggered scheme-III state at its integer time."""
    e = np.zeros(16)
    lib().orc_lf_observe(ctypes.byref(m), _p(_f64(phi)), _p(_f64(pi)), ctypes.c_double(a),
                         ctypes.c_double(b), ctypes.c_double(h), _p(e))
    return _obs_dict(m, e, a)


def Ka(m: Scalar, a, EK, EG, EV) -> float:
    return lib().orc_Ka(ctypes.byref(m), ctypes.c_double(a), ctypes.c_double(EK),
                        ctypes.c_double(EG), ctypes.c_double(EV))


def hc_rhs(m: Scalar, a, rho) -> float:
    return lib().orc_hc_rhs(ctypes.byref(m), ctypes.c_double(a), ctypes.c_double(rho))


# ---------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al. 2011) -- random numbers of the initial state.
# ---------------------------------------------------------------------------
def philox(seed: int, c2: int, c3: int, n: int) -> np.ndarray:
    """(n, 4) uint32 outputs for counters (i, 0..n-1 as 64-bit, c2, c3), key=seed."""
    out = np.empty((n, 4), dtype=np.uint32)
    lib().orc_philox_stream(ctypes.c_uint64(seed), ctypes.c_uint32(c2), ctypes.c_uint32(c3),
                            ctypes.c_int64(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def philox_block(ctr, key) -> tuple:
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(o)


# ---------------------------------------------------------------------------
# Reciprocal lattice (Sec. 3.1)
# ---------------------------------------------------------------------------
def reciprocal(N: int):
    """Integer wave vectors n~ in (-N/2, N/2] for array index 0..N-1, and |n~|."""
    i = np.arange(N)
    nt = np.where(i <= N // 2, i, i - N)
    n1, n2, n3 = np.meshgrid(nt, nt, nt, indexing="ij")
    return n1, n2, n3, np.sqrt(n1 * n1 + n2 * n2 + n3 * n3)


def conjugate_partner(N: int):
    """Linear index of -n~ for every n~, and the linear index itself."""
    i = np.arange(N)
    j = (N - i) % N
    I1, I2, I3 = np.meshgrid(i, i, i, indexing="ij")
    J1, J2, J3 = np.meshgrid(j, j, j, indexing="ij")
    lin = (I1 * N + I2) * N + I3
    par = (J1 * N + J2) * N + J3
    return lin, par


def paper_dft(f: np.ndarray) -> np.ndarray:
    """Forward DFT of Sec. 3.1: f(n~) = sum_n exp(+2 pi i n~.n / N) f(n)."""
    return np.fft.ifftn(f) * f.size


def paper_idft(F: np.ndarray) -> np.ndarray:
    """Inverse DFT of Sec. 3.1: f(n) = N^-3 sum_n~ exp(-2 pi i n~.n / N) f(n~)."""
    return np.fft.fftn(F) / F.size


def potential_curvature(cfg: dict, phibar) -> list:
    """Effective masses m~^2 = d^2 V / d phi_f^2 at the homogeneous values (Sec. 7.1)."""
    m2 = list(cfg.get("m2", (0.0, 0.0))) + [0.0, 0.0]
    lam, q = cfg.get("lam", 0.0), cfg.get("q", 0.0)
    p0 = phibar[0]
    c0 = phibar[1] if len(phibar) > 1 else 0.0
    out = [m2[0] + 3.0 * lam * p0 * p0 + q * c0 * c0]
    if cfg["nf"] > 1:
        out.append(m2[1] + q * p0 * p0)
    return out


def _potential(cfg, phis) -> float:
    m2 = list(cfg.get("m2", (0.0, 0.0))) + [0.0, 0.0]
    lam, q = cfg.get("lam", 0.0), cfg.get("q", 0.0)
    p = phis[0]
    v = 0.5 * m2[0] * p * p + 0.25 * lam * p ** 4
    if cfg["nf"] > 1:
        c = phis[1]
        v += 0.5 * m2[1] * c * c + 0.5 * q * p * p * c * c
    return v


def vacuum_modes(cfg: dict, field: int, m2eff: float, Hhom: float, a: float = 1.0):
    """Fourier modes of the vacuum fluctuation of one real field (Sec. 7.1).

    For every representative of a {n~, -n~} pair (the one with the smaller
    linear index) two Rayleigh moduli |l|, |r| with E|.|^2 = P(k) and two
    uniform phases are drawn from Philox(counter=(lin, field, 0), key=seed):
        P(k) = (w*/f*)^2 (N/dx)^3 / (2 a^2 w_k),  w_k = sqrt(k^2 + a^2 m^2),
        df(n~)  = (|l| e^{i th_l} + |r| e^{i th_r}) / sqrt(2)
        df'(n~) = a^{-(1-alpha)} i w_k (|l| e^{i th_l} - |r| e^{i th_r}) / sqrt(2) - H df(n~)
    The partner gets the complex conjugate; the zero mode and the
    self-conjugate Nyquist corners carry no fluctuation.
    """
    N = int(cfg["N"])
    kIR = float(cfg["kIR"])
    dx = lattice_dx(N, kIR)
    alpha = float(cfg.get("alpha", 1.0))
    w2 = float(cfg.get("omega_over_f", 1.0)) ** 2
    _, _, _, nabs = reciprocal(N)
    k = kIR * nabs
    lin, par = conjugate_partner(N)
    rep = lin < par
    om2 = k * k + a * a * m2eff
    ok = rep & (om2 > 0)
    kcut = float(cfg.get("kcut", 0.0) or 0.0)
    if kcut > 0:
        ok &= k <= kcut
    om = np.sqrt(np.where(ok, om2, 1.0))
    P = np.where(ok, w2 * (N / dx) ** 3 / (2.0 * a * a * om), 0.0)
    u = philox(int(cfg["seed"]), field, 0, N ** 3).reshape(N, N, N, 4).astype(np.float64)
    two32 = 4294967296.0
    ul = (u[..., 0] + 0.5) / two32
    ur = (u[..., 1] + 0.5) / two32
    tl = 2.0 * math.pi * (u[..., 2] + 0.5) / two32
    tr = 2.0 * math.pi * (u[..., 3] + 0.5) / two32
    Rl = np.sqrt(-P * np.log(ul))
    Rr = np.sqrt(-P * np.log(ur))
    L = Rl * np.exp(1j * tl)
    R = Rr * np.exp(1j * tr)
    F = np.where(ok, (L + R) / math.sqrt(2.0), 0.0)
    Fd = np.where(ok, a ** (-(1.0 - alpha)) * 1j * om * (L - R) / math.sqrt(2.0) - Hhom * (L + R) / math.sqrt(2.0), 0.0)
    # Hermitian completion: f(-n~) = conj f(n~)
    Ff = F.ravel().copy()
    Fdf = Fd.ravel().copy()
    linf, parf, okf = lin.ravel(), par.ravel(), ok.ravel()
    Ff[parf[okf]] = np.conj(Ff[linf[okf]])
    Fdf[parf[okf]] = np.conj(Fdf[linf[okf]])
    return Ff.reshape(N, N, N), Fdf.reshape(N, N, N)


def vacuum_ic(cfg: dict) -> dict:
    """Initial state: homogeneous values plus vacuum fluctuations (Sec. 7.1).

    a_0 = 1.  The Hubble rate used inside df' is the homogeneous one; b_0 is then
    fixed from the Hubble constraint with the full lattice energies.  Returns
    synchronised FP64 arrays phi, pi (shape (nf, N, N, N)) and a, b.
    """
    N, nf = int(cfg["N"]), int(cfg["nf"])
    alpha = float(cfg.get("alpha", 1.0))
    a = float(cfg.get("a0", 1.0))
    fmp2 = float(cfg.get("fstar_over_mp", 1.0)) ** 2
    expand = bool(cfg.get("expansion", True))
    phibar = list(cfg.get("phi0", (1.0, 0.0)))[:nf]
    dphibar = list(cfg.get("dphi0", (0.0, 0.0)))[:nf]
    rho_hom = sum(d * d for d in dphibar) / (2.0 * a ** (2 * alpha)) + _potential(cfg, phibar + [0.0])
    Hhom = math.sqrt(fmp2 / 3.0 * a ** (2 * (alpha + 1)) * rho_hom) / a if expand else 0.0
    m2eff = potential_curvature(cfg, phibar + [0.0])
    phi = np.empty((nf, N, N, N))
    pi = np.empty((nf, N, N, N))
    fluct = cfg.get("ic", "vacuum") == "vacuum"
    for f in range(nf):
        if fluct:
            F, Fd = vacuum_modes(cfg, f, m2eff[f], Hhom, a)
            dphi = paper_idft(F).real
            ddphi = paper_idft(Fd).real
        else:
            dphi = ddphi = 0.0
        phi[f] = phibar[f] + dphi
        pi[f] = a ** (3.0 - alpha) * (dphibar[f] + ddphi)
    m = scalar_model(cfg)
    b = 0.0
    if expand:
        o = sync_observe(m, phi, pi, a, 1.0)
        b = math.sqrt(hc_rhs(m, a, o["rho"]))
    return {"phi": phi, "pi": pi, "a": a, "b": b}


# ---------------------------------------------------------------------------
# Power spectrum (Sec. 3.1 discrete spectrum; Sec. 4.4.2)
# ---------------------------------------------------------------------------
def spectrum(f: np.ndarray, kIR: float) -> dict:
    """Radially binned spectrum of a real lattice field.

    Shell b holds the modes with floor(|n~|) = b.  Returned per shell: count,
    S_b = sum |f(n~)|^2, mean k, and
      delta[b]     = (kIR b)^3/(2 pi^2) (dx/N)^3 S_b / (4 pi b^2)   (b >= 1),
                     the paper's angular average normalised by 4 pi |n~|^2;
      delta_avg[b] = kbar_b^3/(2 pi^2) (dx/N)^3 S_b / count_b,
                     the same with the average over the modes in the shell.
    """
    N = f.shape[0]
    dx = lattice_dx(N, kIR)
    F = paper_dft(np.asarray(f, dtype=np.float64))
    P = np.abs(F) ** 2
    _, _, _, nabs = reciprocal(N)
    n1, n2, n3, _ = reciprocal(N)
    b = np.floor(np.sqrt((n1 * n1 + n2 * n2 + n3 * n3).astype(np.float64))).astype(np.int64)
    nb = int(math.floor(math.sqrt(3.0) * N / 2.0)) + 1
    cnt = np.bincount(b.ravel(), minlength=nb)[:nb]
    S = np.bincount(b.ravel(), weights=P.ravel(), minlength=nb)[:nb]
    ksum = np.bincount(b.ravel(), weights=(kIR * nabs).ravel(), minlength=nb)[:nb]
    kbar = np.where(cnt > 0, ksum / np.maximum(cnt, 1), 0.0)
    bb = np.arange(nb, dtype=np.float64)
    norm = (dx / N) ** 3 / (2.0 * math.pi ** 2)
    delta = np.zeros(nb)
    delta[1:] = (kIR * bb[1:]) ** 3 * norm * S[1:] / (4.0 * math.pi * bb[1:] ** 2)
    delta_avg = np.where(cnt > 0, kbar ** 3 * norm * S / np.maximum(cnt, 1), 0.0)
    return {"count": cnt, "S": S, "k": kbar, "delta": delta, "delta_avg": delta_avg}


def _renorm(sp: dict, kIR: float) -> dict:
    S, cnt, kbar = sp["S"], sp["count"], sp["k"]
    N = sp["N"]
    dx = lattice_dx(N, kIR)
    nb = len(S)
    bb = np.arange(nb, dtype=np.float64)
    norm = (dx / N) ** 3 / (2.0 * math.pi ** 2)
    sp["delta"] = np.zeros(nb)
    sp["delta"][1:] = (kIR * bb[1:]) ** 3 * norm * S[1:] / (4.0 * math.pi * bb[1:] ** 2)
    sp["delta_avg"] = np.where(cnt > 0, kbar ** 3 * norm * S / np.maximum(cnt, 1), 0.0)
    return sp


def u1_magnetic_field(cfg: dict, links: np.ndarray) -> np.ndarray:
    """Magnetic field of the U(1) model on the sites (Sec. 5.4 observables),
    B_i for (i, j, k) cyclic:
      compact:      B_i = Im V_jk / (e dx^2), with the plaquette
                    V_jk(n) = V_j(n) V_k(n+j) conj V_j(n+k) conj V_k(n);
      non-compact:  B_i = sum_jk eps_ijk D+_j A_k = D+_j A_k - D+_k A_j.
    The factor i printed before Im V_jk is read as a typo (B is real)."""
    N = int(cfg["N"])
    dx = lattice_dx(N, cfg["kIR"])
    e = float(cfg["e"])
    B = np.empty((3, N, N, N))
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        if cfg.get("model") == "u1nc":
            A = links
            B[i] = ((np.roll(A[k], -1, axis=j) - A[k]) - (np.roll(A[j], -1, axis=k) - A[j])) / dx
        else:
            V = links[:, 0] + 1j * links[:, 1]
            P = V[j] * np.roll(V[k], -1, axis=j) * np.conj(np.roll(V[j], -1, axis=k)) * np.conj(V[k])
            B[i] = P.imag / (e * dx * dx)
    return B


def u1_spectrum(cfg: dict, st: dict, which: str) -> dict:
    """Spectra of the U(1) model (Sec. 5.4.2), binned as spectrum():
      "phi": |Re phi(n~)|^2 + |Im phi(n~)|^2,  "pi": the same for pi_phi,
      "E":   sum_i |E_i(n~)|^2 with E_i = pi_A,i / a^{1-alpha},
      "B":   sum_i |B_i(n~)|^2 with B_i from u1_magnetic_field.
    For "E" the scale factor is st["a"]."""
    kIR = float(cfg["kIR"])
    if which == "phi":
        fields = [st["phi"][0], st["phi"][1]]
    elif which == "pi":
        fields = [st["pi"][0], st["pi"][1]]
    elif which == "E":
        c = st["a"] ** (-(1.0 - float(cfg.get("alpha", 1.0))))
        fields = [c * st["piA"][i] for i in range(3)]
    elif which == "B":
        Bf = u1_magnetic_field(cfg, st["links"])
        fields = [Bf[i] for i in range(3)]
    else:
        raise ValueError(which)
    parts = [spectrum(f, kIR) for f in fields]
    out = {k: v.copy() for k, v in parts[0].items()}
    for p in parts[1:]:
        out["S"] = out["S"] + p["S"]
    out["N"] = fields[0].shape[0]
    return _renorm(out, kIR)


def logk_grid(N: int, kIR: float, nk: int = 64) -> np.ndarray:
    """nk log-spaced wavenumbers from kIR to kIR floor(sqrt(3) N / 2), the
    lowest and highest shells of the lattice (Sec. 3.1 binning)."""
    kmax = kIR * math.floor(math.sqrt(3.0) * N / 2.0)
    return kIR * (kmax / kIR) ** (np.arange(nk, dtype=np.float64) / (nk - 1))


def log_interp(kbar: np.ndarray, value: np.ndarray, valid: np.ndarray, kq: np.ndarray) -> np.ndarray:
    """log10(value) interpolated linearly in log10 k between the valid shell
    centres kbar, held constant beyond the first and last valid shell."""
    xs, ys = [], []
    for b in range(len(kbar)):
        if valid[b]:
            xs.append(math.log10(kbar[b]))
            ys.append(math.log10(value[b]))
    out = np.empty(len(kq))
    for j, k in enumerate(kq):
        x = math.log10(k)
        if x <= xs[0]:
            out[j] = ys[0]
        elif x >= xs[-1]:
            out[j] = ys[-1]
        else:
            i = 0
            while xs[i + 1] < x:
                i += 1
            t = (x - xs[i]) / (xs[i + 1] - xs[i])
            out[j] = ys[i] + t * (ys[i + 1] - ys[i])
    return out


def spectrum_logk(f: np.ndarray, kIR: float, nk: int = 64) -> np.ndarray:
    """The surrogate's target: log10 of the mode-averaged spectrum
    delta_avg (shells b >= 1 with modes and positive power) at the nk
    wavenumbers of logk_grid."""
    s = spectrum(f, kIR)
    b = np.arange(len(s["count"]))
    valid = (b >= 1) & (s["count"] > 0) & (s["delta_avg"] > 0)
    return log_interp(s["k"], s["delta_avg"], valid, logk_grid(f.shape[0], kIR, nk))


# ---------------------------------------------------------------------------
# Complex scalar with compact U(1) links (Sec. 5.1, 5.3, 5.4; ICs Sec. 7.2)
# ---------------------------------------------------------------------------
class U1(ctypes.Structure):
    """Parameters of the Abelian-Higgs model (compact links, or with
    noncompact = 1 the real gauge field A_i of Sec. 5.2)."""
    _fields_ = [("N", ctypes.c_int32), ("expand", ctypes.c_int32), ("noncompact", ctypes.c_int32),
                ("pad1", ctypes.c_int32), ("dx", ctypes.c_double), ("alpha", ctypes.c_double),
                ("fmp2", ctypes.c_double), ("lam", ctypes.c_double), ("m2", ctypes.c_double),
                ("e", ctypes.c_double), ("wf2", ctypes.c_double)]


def u1_model(cfg: dict) -> U1:
    m = U1()
    m.N = int(cfg["N"])
    m.expand = 1 if cfg.get("expansion", True) else 0
    m.noncompact = 1 if cfg.get("model") == "u1nc" else 0
    m.dx = lattice_dx(m.N, cfg["kIR"])
    m.alpha = float(cfg.get("alpha", 1.0))
    m.fmp2 = float(cfg.get("fstar_over_mp", 1.0)) ** 2
    m.lam = float(cfg.get("lam", 0.0))
    m.m2 = float(list(cfg.get("m2", (0.0, 0.0)))[0])
    m.e = float(cfg["e"])
    m.wf2 = float(cfg.get("omega_over_f", 1.0)) ** 2
    return m


def u1_kernels(m: U1, a, phi, links):
    Kp = np.empty_like(phi)
    KA = np.empty((3,) + phi.shape[1:])
    lib().orc_u1_kernels(ctypes.byref(m), ctypes.c_double(a), _p(_f64(phi)), _p(_f64(links)), _p(Kp), _p(KA))
    return Kp, KA


def u1_lf_startup(m: U1, st: dict, h: float):
    ca, cb = ctypes.c_double(st["a"]), ctypes.c_double(st["b"])
    lib().orc_u1_lf_startup(ctypes.byref(m), _p(st["phi"]), _p(st["pi"]), _p(st["links"]), _p(st["piA"]),
                            ctypes.byref(ca), ctypes.byref(cb), ctypes.c_double(h))
    st["a"], st["b"] = ca.value, cb.value


def u1_lf_steps(m: U1, st: dict, h: float, nsteps: int, omp: bool = False):
    """nsteps compact staggered-leapfrog steps (Sec. 5.3.1), in place on st."""
    ca, cb = ctypes.c_double(st["a"]), ctypes.c_double(st["b"])
    lib(omp).orc_u1_lf_steps(ctypes.byref(m), _p(st["phi"]), _p(st["pi"]), _p(st["links"]), _p(st["piA"]),
                             ctypes.byref(ca), ctypes.byref(cb), ctypes.c_double(h), ctypes.c_int64(nsteps))
    st["a"], st["b"] = ca.value, cb.value


def u1_vv_steps(m: U1, st: dict, h: float, integrator: str = "vv2", nsteps: int = 1, omp: bool = False):
    """nsteps compact velocity-Verlet steps (Sec. 5.3.2; Yoshida VVn, Sec. 5.3.3)
    of a synchronised state, in place on st."""
    w = np.ascontiguousarray(VV_WEIGHTS[integrator], dtype=np.float64)
    ca, cb = ctypes.c_double(st["a"]), ctypes.c_double(st["b"])
    lib(omp).orc_u1_vv_steps(ctypes.byref(m), _p(st["phi"]), _p(st["pi"]), _p(st["links"]), _p(st["piA"]),
                             ctypes.byref(ca), ctypes.byref(cb), ctypes.c_double(h), _p(w), ctypes.c_int(len(w)),
                             ctypes.c_int64(nsteps))
    st["a"], st["b"] = ca.value, cb.value


def _u1_obs(e, a):
    d = {"a": a, "EK": e[0], "EG": e[1], "EV": e[2], "EK_A": e[3], "EG_A": e[4], "EV_quartic": e[5],
         "EV_mass": e[6], "b": e[7], "hc": e[8], "gauss": e[9], "mean0": e[10], "mean1": e[11],
         "meansq": e[12]}
    d["rho"] = e[0] + e[1] + e[2] + e[3] + e[4]
    d["p"] = e[0] - e[1] / 3.0 - e[2] + (e[3] + e[4]) / 3.0
    d["w"] = d["p"] / d["rho"] if d["rho"] != 0 else 0.0
    return d


def u1_lf_observe(m: U1, st: dict, h: float) -> dict:
    e = np.zeros(13)
    lib().orc_u1_lf_observe(ctypes.byref(m), _p(st["phi"]), _p(st["pi"]), _p(st["links"]), _p(st["piA"]),
                            ctypes.c_double(st["a"]), ctypes.c_double(st["b"]), ctypes.c_double(h), _p(e))
    return _u1_obs(e, st["a"])


def u1_sync_observe(m: U1, st: dict) -> dict:
    e = np.zeros(13)
    lib().orc_u1_sync_observe(ctypes.byref(m), _p(st["phi"]), _p(st["pi"]), _p(st["links"]), _p(st["piA"]),
                              ctypes.c_double(st["a"]), ctypes.c_double(st["b"]), _p(e))
    return _u1_obs(e, st["a"])


def u1_gauss(m: U1, st: dict) -> np.ndarray:
    out = np.zeros(4)
    lib().orc_u1_gauss(ctypes.byref(m), _p(st["phi"]), _p(st["pi"]), _p(st["piA"]), _p(out))
    return out


def u1_potential(cfg, phibar) -> float:
    """V = lambda |phi|^4 + m2 |phi|^2 with |phi|^2 = (phi_0^2 + phi_1^2)/2."""
    r2 = 0.5 * (phibar[0] ** 2 + phibar[1] ** 2)
    return float(cfg.get("lam", 0.0)) * r2 * r2 + float(list(cfg.get("m2", (0.0, 0.0)))[0]) * r2


def u1_vacuum_ic(cfg: dict) -> dict:
    """Initial state of the compact U(1) model (Sec. 7.2).

    Real components phi_0, phi_1 of phi = (phi_0 + i phi_1)/sqrt 2 get the
    vacuum modes of Sec. 7.1 with the constraints that remove the zero mode of
    the charge: |l_n| = |r_n| and th_1^r = th_0^r + th_1^l - th_0^l.  Random
    numbers: Philox(counter=(lin, n, 0), key=seed); u0 -> |l_n|, u2 -> th_n^l,
    u3 of component 0 -> th_0^r.  Links V = 1 (A = 0); the link momenta solve
    the discrete Gauss law sum_i Delta^-_i piA_i = rho in Fourier space with
    the minimum-norm solution E_i = conj(s_i) rho / sum_j |s_j|^2,
    s_j = (1 - exp(+2 pi i n~_j / N)) / dx; b_0 from the Hubble constraint.
    For the non-compact model ("model": "u1nc") "links" holds A_i = 0,
    shape (3, N, N, N); compact links are (Re, Im) pairs, shape (3, 2, N, N, N).
    """
    N = int(cfg["N"])
    kIR = float(cfg["kIR"])
    dx = lattice_dx(N, kIR)
    alpha = float(cfg.get("alpha", 1.0))
    a = float(cfg.get("a0", 1.0))
    w2 = float(cfg.get("omega_over_f", 1.0)) ** 2
    e = float(cfg["e"])
    lam = float(cfg.get("lam", 0.0))
    m2 = float(list(cfg.get("m2", (0.0, 0.0)))[0])
    fmp2 = float(cfg.get("fstar_over_mp", 1.0)) ** 2
    expand = bool(cfg.get("expansion", True))
    pb = list(cfg.get("phi0", (1.0, 0.0)))[:2]
    db = list(cfg.get("dphi0", (0.0, 0.0)))[:2]
    rho_hom = (db[0] ** 2 + db[1] ** 2) / (2.0 * a ** (2 * alpha)) + u1_potential(cfg, pb)
    Hh = math.sqrt(fmp2 / 3.0 * a ** (2 * (alpha + 1)) * rho_hom) / a if expand else 0.0
    s = pb[0] ** 2 + pb[1] ** 2
    m2eff = [lam * (s + 2.0 * pb[n] ** 2) + m2 for n in range(2)]
    n1, n2, n3, nabs = reciprocal(N)
    k = kIR * nabs
    lin, par = conjugate_partner(N)
    rep = lin < par
    kcut = float(cfg.get("kcut", 0.0) or 0.0)
    two32 = 4294967296.0
    U = [philox(int(cfg["seed"]), n, 0, N ** 3).reshape(N, N, N, 4).astype(np.float64) for n in range(2)]
    th_l = [2.0 * math.pi * (U[n][..., 2] + 0.5) / two32 for n in range(2)]
    th0r = 2.0 * math.pi * (U[0][..., 3] + 0.5) / two32
    th_r = [th0r, th0r + th_l[1] - th_l[0]]
    fields, derivs = [], []
    for n in range(2):
        om2 = k * k + a * a * m2eff[n]
        ok = rep & (om2 > 0)
        if kcut > 0:
            ok &= k <= kcut
        om = np.sqrt(np.where(ok, om2, 1.0))
        P = np.where(ok, w2 * (N / dx) ** 3 / (2.0 * a * a * om), 0.0)
        R = np.sqrt(-P * np.log((U[n][..., 0] + 0.5) / two32))
        L = R * np.exp(1j * th_l[n])
        Rt = R * np.exp(1j * th_r[n])
        F = np.where(ok, (L + Rt) / math.sqrt(2.0), 0.0).ravel()
        Fd = np.where(ok, a ** (-(1.0 - alpha)) * 1j * om * (L - Rt) / math.sqrt(2.0)
                      - Hh * (L + Rt) / math.sqrt(2.0), 0.0).ravel()
        okf, linf, parf = ok.ravel(), lin.ravel(), par.ravel()
        F[parf[okf]] = np.conj(F[linf[okf]])
        Fd[parf[okf]] = np.conj(Fd[linf[okf]])
        fields.append(pb[n] + paper_idft(F.reshape(N, N, N)).real)
        derivs.append(db[n] + paper_idft(Fd.reshape(N, N, N)).real)
    r2 = 1.0 / math.sqrt(2.0)
    phi = np.stack([fields[0] * r2, fields[1] * r2])
    pi = a ** (3.0 - alpha) * np.stack([derivs[0] * r2, derivs[1] * r2])
    rho = 2.0 * e / w2 * (phi[0] * pi[1] - phi[1] * pi[0])
    Rh = paper_dft(rho)
    sj = [(1.0 - np.exp(2j * math.pi * nn / N)) / dx for nn in (n1, n2, n3)]
    den = sum(np.abs(x) ** 2 for x in sj)
    zero = den == 0
    # The leapfrog and Verlet kicks conserve G = sum_i D-_i piA_i - rho(phi, pi)
    # exactly, with no power of a in it (Sec. 5.3 kernels), so the link momenta
    # themselves solve the discrete Gauss law for any a0 and alpha.
    piA = np.stack([paper_idft(np.where(zero, 0.0, np.conj(x) * Rh / np.where(zero, 1.0, den))).real
                    for x in sj])
    if cfg.get("model") == "u1nc":
        links = np.zeros((3, N, N, N))
    else:
        links = np.zeros((3, 2, N, N, N))
        links[:, 0] = 1.0
    st = {"phi": phi, "pi": pi, "links": links, "piA": piA, "a": a, "b": 1.0}
    if expand:
        o = u1_sync_observe(u1_model(cfg), st)
        st["b"] = math.sqrt(fmp2 / 3.0 * a ** (2 * (alpha + 1)) * o["rho"])
    else:
        st["b"] = 0.0
    return st


# ---------------------------------------------------------------------------
# Doublet with SU(2) x U(1) links (Sec. 6; ICs Sec. 7.2)
# ---------------------------------------------------------------------------
class SU2(ctypes.Structure):
    """Parameters of the SU(2) x U(1) doublet model: V = lam |Phi|^4 + m2 |Phi|^2,
    U(1) coupling e = g_A Q_A, SU(2) coupling g = g_B Q_B."""
    _fields_ = [("N", ctypes.c_int32), ("expand", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("pad1", ctypes.c_int32), ("dx", ctypes.c_double), ("alpha", ctypes.c_double),
                ("fmp2", ctypes.c_double), ("lam", ctypes.c_double), ("m2", ctypes.c_double),
                ("e", ctypes.c_double), ("g", ctypes.c_double), ("wf2", ctypes.c_double)]


def su2_model(cfg: dict) -> SU2:
    m = SU2()
    m.N = int(cfg["N"])
    m.expand = 1 if cfg.get("expansion", True) else 0
    m.dx = lattice_dx(m.N, cfg["kIR"])
    m.alpha = float(cfg.get("alpha", 1.0))
    m.fmp2 = float(cfg.get("fstar_over_mp", 1.0)) ** 2
    m.lam = float(cfg.get("lam", 0.0))
    m.m2 = float(list(cfg.get("m2", (0.0, 0.0)))[0])
    m.e = float(cfg["e"])
    m.g = float(cfg["g"])
    m.wf2 = float(cfg.get("omega_over_f", 1.0)) ** 2
    return m


def _su2_args(st):
    return (_p(st["phi"]), _p(st["pi"]), _p(st["links"]), _p(st["su2"]), _p(st["piA"]), _p(st["piB"]))


def su2_kernels(m: SU2, a, st):
    N = m.N
    Kp, KA, KB = np.empty((4, N, N, N)), np.empty((3, N, N, N)), np.empty((3, 3, N, N, N))
    lib().orc_su2_kernels(ctypes.byref(m), ctypes.c_double(a), _p(st["phi"]), _p(st["links"]), _p(st["su2"]),
                          _p(Kp), _p(KA), _p(KB))
    return Kp, KA, KB


def su2_lf_startup(m: SU2, st: dict, h: float):
    ca, cb = ctypes.c_double(st["a"]), ctypes.c_double(st["b"])
    lib().orc_su2_lf_startup(ctypes.byref(m), *_su2_args(st), ctypes.byref(ca), ctypes.byref(cb), ctypes.c_double(h))
    st["a"], st["b"] = ca.value, cb.value


def su2_lf_steps(m: SU2, st: dict, h: float, nsteps: int, omp: bool = False):
    """nsteps SU(N) staggered-leapfrog steps (Sec. 6.2.1), in place on st."""
    ca, cb = ctypes.c_double(st["a"]), ctypes.c_double(st["b"])
    lib(omp).orc_su2_lf_steps(ctypes.byref(m), *_su2_args(st), ctypes.byref(ca), ctypes.byref(cb),
                              ctypes.c_double(h), ctypes.c_int64(nsteps))
    st["a"], st["b"] = ca.value, cb.value


def su2_vv_steps(m: SU2, st: dict, h: float, integrator: str = "vv2", nsteps: int = 1, omp: bool = False):
    """nsteps velocity-Verlet / Yoshida steps (Sec. 6.2.2, 6.2.3), in place on st."""
    w = np.ascontiguousarray(VV_WEIGHTS[integrator], dtype=np.float64)
    ca, cb = ctypes.c_double(st["a"]), ctypes.c_double(st["b"])
    lib(omp).orc_su2_vv_steps(ctypes.byref(m), *_su2_args(st), ctypes.byref(ca), ctypes.byref(cb),
                              ctypes.c_double(h), _p(w), ctypes.c_int(len(w)), ctypes.c_int64(nsteps))
    st["a"], st["b"] = ca.value, cb.value


def _su2_obs(e, a):
    d = {"a": a, "EK": e[0], "EG": e[1], "EV": e[2], "EK_A": e[3], "EG_A": e[4], "EK_B": e[5], "EG_B": e[6],
         "EV_quartic": e[7], "EV_mass": e[8], "b": e[9], "hc": e[10], "gauss": e[11], "gauss_B": e[12],
         "mean": [e[13], e[14], e[15], e[16]], "meansq": e[17]}
    d["rho"] = sum(e[k] for k in range(7))
    d["p"] = e[0] - e[1] / 3.0 - e[2] + (e[3] + e[4] + e[5] + e[6]) / 3.0
    d["w"] = d["p"] / d["rho"] if d["rho"] != 0 else 0.0
    return d


def su2_lf_observe(m: SU2, st: dict, h: float) -> dict:
    e = np.zeros(18)
    lib().orc_su2_lf_observe(ctypes.byref(m), *_su2_args(st), ctypes.c_double(st["a"]), ctypes.c_double(st["b"]),
                             ctypes.c_double(h), _p(e))
    return _su2_obs(e, st["a"])


def su2_sync_observe(m: SU2, st: dict) -> dict:
    e = np.zeros(18)
    lib().orc_su2_sync_observe(ctypes.byref(m), *_su2_args(st), ctypes.c_double(st["a"]), ctypes.c_double(st["b"]),
                               _p(e))
    return _su2_obs(e, st["a"])


def su2_gauss(m: SU2, st: dict) -> np.ndarray:
    out = np.zeros(10)
    lib().orc_su2_gauss(ctypes.byref(m), _p(st["phi"]), _p(st["pi"]), _p(st["su2"]), _p(st["piA"]), _p(st["piB"]),
                        _p(out))
    return out


def su2_charges(cfg: dict, phi: np.ndarray, pi: np.ndarray):
    """Charge densities of the doublet (Sec. 6.2 Gauss laws):
    rho_A = 2e (f/w)^2 Im[Phi^dag pi],  rho_B^a = g (f/w)^2 Im[Phi^dag sigma_a pi]."""
    w2 = float(cfg.get("omega_over_f", 1.0)) ** 2
    P = [phi[0] + 1j * phi[1], phi[2] + 1j * phi[3]]
    Q = [pi[0] + 1j * pi[1], pi[2] + 1j * pi[3]]
    rhoA = 2.0 * float(cfg["e"]) / w2 * (np.conj(P[0]) * Q[0] + np.conj(P[1]) * Q[1]).imag
    s = [np.conj(P[0]) * Q[1] + np.conj(P[1]) * Q[0],                 # Phi^dag sigma_1 pi
         -1j * np.conj(P[0]) * Q[1] + 1j * np.conj(P[1]) * Q[0],       # Phi^dag sigma_2 pi
         np.conj(P[0]) * Q[0] - np.conj(P[1]) * Q[1]]                  # Phi^dag sigma_3 pi
    rhoB = np.stack([float(cfg["g"]) / w2 * x.imag for x in s])
    return rhoA, rhoB


def _gauss_solve(rho: np.ndarray, N: int, dx: float) -> np.ndarray:
    """Minimum-norm solution E_i of sum_i D-_i E_i = rho (Sec. 7.2):
    E_i(n~) = conj(s_i) rho(n~) / sum_j |s_j|^2, s_j = (1 - exp(+2 pi i n~_j/N))/dx, E(0) = 0."""
    n1, n2, n3, _ = reciprocal(N)
    Rh = paper_dft(rho)
    sj = [(1.0 - np.exp(2j * math.pi * nn / N)) / dx for nn in (n1, n2, n3)]
    den = sum(np.abs(x) ** 2 for x in sj)
    zero = den == 0
    return np.stack([paper_idft(np.where(zero, 0.0, np.conj(x) * Rh / np.where(zero, 1.0, den))).real for x in sj])


def su2_vacuum_ic(cfg: dict) -> dict:
    """Initial state of the SU(2) x U(1) doublet (Sec. 7.2).

    Real components phi_n (n = 0..3) of Phi = (phi_0 + i phi_1, phi_2 + i phi_3)/sqrt 2
    get the homogeneous values phi0[n] plus vacuum modes (Sec. 7.1) with
    |l_n| = |r_n| and th_m^r = th_0^r + th_m^l - th_0^l (m = 1, 2, 3); with equal
    homogeneous values (equal effective masses) every charge then vanishes mode by
    mode.  Random numbers: Philox(counter=(lin, n, 0), key=seed); u0 -> |l_n|,
    u2 -> th_n^l, u3 of component 0 -> th_0^r.  Links V = 1 and U = 1 (A = B = 0);
    the electric fields solve both Gauss laws with the minimum-norm Fourier
    solution; b from the Hubble constraint.  Shapes: phi, pi (4, N, N, N); links
    (3, 2, N, N, N); su2 (3, 4, N, N, N) as (c0, c1, c2, c3); piA (3, N, N, N);
    piB (3, 3, N, N, N)."""
    N = int(cfg["N"])
    kIR = float(cfg["kIR"])
    dx = lattice_dx(N, kIR)
    alpha = float(cfg.get("alpha", 1.0))
    a = float(cfg.get("a0", 1.0))
    w2 = float(cfg.get("omega_over_f", 1.0)) ** 2
    lam = float(cfg.get("lam", 0.0))
    m2 = float(list(cfg.get("m2", (0.0, 0.0)))[0])
    fmp2 = float(cfg.get("fstar_over_mp", 1.0)) ** 2
    expand = bool(cfg.get("expansion", True))
    pb = list(cfg.get("phi0", (0.5, 0.5, 0.5, 0.5)))
    db = list(cfg.get("dphi0", (0.0, 0.0, 0.0, 0.0)))
    s = sum(x * x for x in pb)
    r2 = 0.5 * s
    rho_hom = sum(x * x for x in db) / (2.0 * a ** (2 * alpha)) + lam * r2 * r2 + m2 * r2
    Hh = math.sqrt(fmp2 / 3.0 * a ** (2 * (alpha + 1)) * rho_hom) / a if expand else 0.0
    m2eff = [lam * (s + 2.0 * pb[n] ** 2) + m2 for n in range(4)]
    _, _, _, nabs = reciprocal(N)
    k = kIR * nabs
    lin, par = conjugate_partner(N)
    rep = lin < par
    kcut = float(cfg.get("kcut", 0.0) or 0.0)
    two32 = 4294967296.0
    U = [philox(int(cfg["seed"]), n, 0, N ** 3).reshape(N, N, N, 4).astype(np.float64) for n in range(4)]
    th_l = [2.0 * math.pi * (U[n][..., 2] + 0.5) / two32 for n in range(4)]
    th0r = 2.0 * math.pi * (U[0][..., 3] + 0.5) / two32
    th_r = [th0r] + [th0r + th_l[n] - th_l[0] for n in range(1, 4)]
    fields, derivs = [], []
    for n in range(4):
        om2 = k * k + a * a * m2eff[n]
        ok = rep & (om2 > 0)
        if kcut > 0:
            ok &= k <= kcut
        om = np.sqrt(np.where(ok, om2, 1.0))
        P = np.where(ok, w2 * (N / dx) ** 3 / (2.0 * a * a * om), 0.0)
        R = np.sqrt(-P * np.log((U[n][..., 0] + 0.5) / two32))
        L = R * np.exp(1j * th_l[n])
        Rt = R * np.exp(1j * th_r[n])
        F = np.where(ok, (L + Rt) / math.sqrt(2.0), 0.0).ravel()
        Fd = np.where(ok, a ** (-(1.0 - alpha)) * 1j * om * (L - Rt) / math.sqrt(2.0)
                      - Hh * (L + Rt) / math.sqrt(2.0), 0.0).ravel()
        okf, linf, parf = ok.ravel(), lin.ravel(), par.ravel()
        F[parf[okf]] = np.conj(F[linf[okf]])
        Fd[parf[okf]] = np.conj(Fd[linf[okf]])
        fields.append(pb[n] + paper_idft(F.reshape(N, N, N)).real)
        derivs.append(db[n] + paper_idft(Fd.reshape(N, N, N)).real)
    r = 1.0 / math.sqrt(2.0)
    phi = np.stack([f * r for f in fields])
    pi = a ** (3.0 - alpha) * np.stack([d * r for d in derivs])
    rhoA, rhoB = su2_charges(cfg, phi, pi)
    links = np.zeros((3, 2, N, N, N))
    links[:, 0] = 1.0
    su2 = np.zeros((3, 4, N, N, N))
    su2[:, 0] = 1.0
    piA = _gauss_solve(rhoA, N, dx)
    piB = np.stack([_gauss_solve(rhoB[c], N, dx) for c in range(3)], axis=1)   # (i, a, ...)
    st = {"phi": phi, "pi": pi, "links": links, "su2": su2, "piA": np.ascontiguousarray(piA),
          "piB": np.ascontiguousarray(piB), "a": a, "b": 1.0}
    if expand:
        o = su2_sync_observe(su2_model(cfg), st)
        st["b"] = math.sqrt(fmp2 / 3.0 * a ** (2 * (alpha + 1)) * o["rho"])
    else:
        st["b"] = 0.0
    return st
