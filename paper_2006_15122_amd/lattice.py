"""Python binding of the C ABI in include/cosmolat.h (argument marshalling only).

Every step of the method runs in the HIP library libcosmolat.so; this module
only converts configuration dicts and numpy arrays, allocates the device
workspace with torch (the library never allocates device memory) and passes
torch's current HIP stream.  Missing library -> ImportError, loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcosmolat.so")
_LIB = None

LAT_MODEL_SCALAR, LAT_MODEL_U1, LAT_MODEL_U1_NC, LAT_MODEL_SU2U1 = 0, 1, 2, 3
MODELS = {"scalar": LAT_MODEL_SCALAR, "u1": LAT_MODEL_U1, "u1nc": LAT_MODEL_U1_NC, "su2u1": LAT_MODEL_SU2U1}
INTEGRATORS = {"lf2": 0, "vv2": 1, "vv4": 2, "vv6": 3, "vv8": 4, "vv10": 5}
PRECISIONS = {"fp64": 0, "fp32": 1}
ICS = {"vacuum": 0, "homogeneous": 1}
ERRORS = {-1: "LAT_EINVAL", -2: "LAT_ENOMEM", -3: "LAT_EHIP", -4: "LAT_ENONFINITE", -5: "LAT_ESTATE"}

EXPORTS = ["lattice_workspace_size", "lattice_init", "lattice_set_state", "lattice_get_state",
           "lattice_step", "lattice_energies", "lattice_energies_noalloc", "lattice_spectrum", "lattice_spectrum_logk", "lattice_destroy",
           "lattice_last_error", "lattice_get_tiling", "lattice_set_tiling",
           "lattice_field_device_ptr", "lattice_pass_timer", "lattice_pass_timer_read", "lattice_batch_workspace_size", "lattice_batch_init",
           "lattice_batch_step", "lattice_batch_energies", "lattice_batch_run",
           "lattice_batch_get_tiling", "lattice_batch_set_tiling", "lattice_batch_use_graph",
           "lattice_batch_destroy"]


# spectrum selectors of the U(1) models that add components (cosmolat.h)
SPEC_U1_PHI, SPEC_U1_PI, SPEC_U1_E, SPEC_U1_B = 32, 33, 34, 35

class LatticeError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"{ERRORS.get(rc, rc)}: {msg}")
        self.rc = rc


class Params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("nf", ctypes.c_int32), ("N", ctypes.c_int32),
                ("integrator", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("expansion", ctypes.c_int32), ("ic", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("kIR", ctypes.c_double), ("dt", ctypes.c_double),
                ("alpha", ctypes.c_double), ("fstar_over_mp", ctypes.c_double),
                ("omega_over_f", ctypes.c_double), ("m2", ctypes.c_double * 2),
                ("lam", ctypes.c_double), ("q", ctypes.c_double), ("e", ctypes.c_double),
                ("phi0", ctypes.c_double * 2), ("dphi0", ctypes.c_double * 2),
                ("a0", ctypes.c_double), ("kcut", ctypes.c_double), ("g", ctypes.c_double)]


class Scalars(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("eta", ctypes.c_double),
                ("step", ctypes.c_int64), ("staggered", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Obs(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("H", ctypes.c_double), ("EK", ctypes.c_double), ("EG", ctypes.c_double),
                ("EV", ctypes.c_double), ("EV_term", ctypes.c_double * 3),
                ("EK_f", ctypes.c_double * 2), ("EG_f", ctypes.c_double * 2),
                ("mean_f", ctypes.c_double * 2), ("meansq_f", ctypes.c_double * 2),
                ("EK_A", ctypes.c_double), ("EG_A", ctypes.c_double), ("rho", ctypes.c_double),
                ("p", ctypes.c_double), ("w", ctypes.c_double), ("hc", ctypes.c_double),
                ("gauss", ctypes.c_double), ("step", ctypes.c_int64), ("staggered", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("EK_B", ctypes.c_double), ("EG_B", ctypes.c_double),
                ("gauss_B", ctypes.c_double), ("mean_lo", ctypes.c_double * 2)]


def lib():
    """Load libcosmolat.so (built by __graft_entry__.build()).  No fallback."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO):
            raise ImportError(f"HIP library {_SO} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_SO)
        L.lattice_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "lattice_last_error":
                getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(rc):
    if rc != 0:
        raise LatticeError(rc, lib().lattice_last_error().decode())


def params(cfg: dict) -> Params:
    p = Params()
    p.model = MODELS[cfg.get("model", "scalar")]
    p.nf = int(cfg["nf"])
    p.N = int(cfg["N"])
    p.integrator = INTEGRATORS[cfg.get("integrator", "vv2")]
    p.precision = PRECISIONS[cfg.get("precision", "fp32")]
    p.expansion = 1 if cfg.get("expansion", True) else 0
    p.ic = ICS[cfg.get("ic", "vacuum")]
    p.seed = int(cfg.get("seed", 0))
    p.kIR = float(cfg["kIR"])
    p.dt = float(cfg["dt"])
    p.alpha = float(cfg.get("alpha", 1.0))
    p.fstar_over_mp = float(cfg.get("fstar_over_mp", 1.0))
    p.omega_over_f = float(cfg.get("omega_over_f", 1.0))
    m2 = list(cfg.get("m2", (0.0, 0.0))) + [0.0, 0.0]
    p.m2[0], p.m2[1] = float(m2[0]), float(m2[1])
    p.lam = float(cfg.get("lam", 0.0))
    p.q = float(cfg.get("q", 0.0))
    p.e = float(cfg.get("e", 0.0))
    p.g = float(cfg.get("g", 0.0))
    ph = list(cfg.get("phi0", (1.0, 0.0))) + [0.0, 0.0]
    dph = list(cfg.get("dphi0", (0.0, 0.0))) + [0.0, 0.0]
    p.phi0[0], p.phi0[1] = float(ph[0]), float(ph[1])
    p.dphi0[0], p.dphi0[1] = float(dph[0]), float(dph[1])
    p.a0 = float(cfg.get("a0", 1.0))
    p.kcut = float(cfg.get("kcut", 0.0) or 0.0)
    return p


def workspace_size(cfg: dict) -> int:
    n = ctypes.c_size_t()
    _check(lib().lattice_workspace_size(ctypes.byref(params(cfg)), ctypes.byref(n)))
    return n.value


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def obs_dict(o: Obs, nf: int) -> dict:
    d = {k: getattr(o, k) for k in ("eta", "a", "b", "H", "EK", "EG", "EV", "EK_A", "EG_A", "rho",
                                    "p", "w", "hc", "gauss", "step", "staggered", "EK_B", "EG_B", "gauss_B")}
    d["EV_mass"], d["EV_quartic"], d["EV_int"] = o.EV_term[0], o.EV_term[1], o.EV_term[2]
    if nf == 4:
        # the doublet: means of its four real components, <|Phi|^2>
        d["mean"] = [o.mean_f[0], o.mean_f[1], o.mean_lo[0], o.mean_lo[1]]
        d["meansq"] = o.meansq_f[0]
        return d
    for f in range(nf):
        d[f"EK{f}"] = o.EK_f[f]
        d[f"EG{f}"] = o.EG_f[f]
        d[f"mean{f}"] = o.mean_f[f]
        d[f"meansq{f}"] = o.meansq_f[f]
    return d


class Lattice:
    """One lattice on one GPU.  cfg: a workload dict (see synth.py)."""

    def __init__(self, cfg: dict, device: str = "cuda:0", stream=None, ws_fill=None, _handle=None,
                 _owner=None):
        """ws_fill: a byte (0..255) written over the whole workspace before
        lattice_init, so that a test can show no result depends on what the
        memory held (0xFF makes every FP32 and FP64 word a NaN)."""
        self.cfg = dict(cfg)
        self.p = params(cfg)
        self.nf = self.p.nf
        self.N = self.p.N
        if _handle is not None:
            # a run owned by a Batch: no workspace of its own
            self.h = _handle
            self._owner = _owner
            self._borrowed = True
            return
        import torch

        self._borrowed = False
        nbytes = workspace_size(cfg)
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        if ws_fill is not None:
            self.ws.fill_(int(ws_fill))
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = ctypes.c_void_p()
        _check(lib().lattice_init(ctypes.byref(self.p), ctypes.c_void_p(base + off),
                                  ctypes.c_size_t(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(self.h)))

    # -- state --------------------------------------------------------------
    def set_state(self, phi, pi, a, b, eta=0.0, step=0, staggered=False, links=None, piA=None, su2=None,
                  piB=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        pi = np.ascontiguousarray(pi, dtype=np.float64)
        s = Scalars(a=float(a), b=float(b), eta=float(eta), step=int(step),
                    staggered=1 if staggered else 0, reserved=0)
        lk = pa = None
        V = self.N ** 3
        if phi.size != self.nf * V or pi.size != self.nf * V:
            raise ValueError(f"phi and pi must hold {self.nf} x N^3 values")
        if self.p.model == LAT_MODEL_SU2U1:
            # the C ABI takes the U(1) links then the SU(2) links, pi_A then pi_B
            if links is None or su2 is None or piA is None or piB is None:
                raise ValueError("the SU(2) x U(1) state needs links, su2, piA and piB")
            lk = np.ascontiguousarray(np.concatenate([np.ravel(links), np.ravel(su2)]), dtype=np.float64)
            pa = np.ascontiguousarray(np.concatenate([np.ravel(piA), np.ravel(piB)]), dtype=np.float64)
            if lk.size != 18 * V or pa.size != 12 * V:
                raise ValueError("links (3,2,N,N,N), su2 (3,4,N,N,N), piA (3,N,N,N), piB (3,3,N,N,N)")
        elif links is not None:
            lk = np.ascontiguousarray(links, dtype=np.float64)
            pa = np.ascontiguousarray(piA, dtype=np.float64)
            # compact links are (Re, Im) pairs; the non-compact model takes A_i
            want = 3 * V if self.p.model == LAT_MODEL_U1_NC else 6 * V
            if lk.size != want or pa.size != 3 * V:
                raise ValueError(f"links must hold {want} values and piA {3 * V}")
        _check(lib().lattice_set_state(self.h, _dp(phi), _dp(pi), _dp(lk) if lk is not None else None,
                                       _dp(pa) if pa is not None else None, ctypes.byref(s)))

    def get_state(self) -> dict:
        N, nf = self.N, self.nf
        phi = np.empty((nf, N, N, N))
        pi = np.empty((nf, N, N, N))
        s = Scalars()
        links = piA = None
        if self.p.model == LAT_MODEL_U1:
            links = np.empty((3, 2, N, N, N))
            piA = np.empty((3, N, N, N))
        elif self.p.model == LAT_MODEL_U1_NC:
            links = np.empty((3, N, N, N))
            piA = np.empty((3, N, N, N))
        elif self.p.model == LAT_MODEL_SU2U1:
            links = np.empty(18 * N ** 3)
            piA = np.empty(12 * N ** 3)
        _check(lib().lattice_get_state(self.h, _dp(phi), _dp(pi), _dp(links) if links is not None else None,
                                       _dp(piA) if piA is not None else None, ctypes.byref(s)))
        out = {"phi": phi, "pi": pi, "a": s.a, "b": s.b, "eta": s.eta, "step": s.step,
               "staggered": bool(s.staggered)}
        if self.p.model == LAT_MODEL_SU2U1:
            V = N ** 3
            out["links"] = links[:6 * V].reshape(3, 2, N, N, N)
            out["su2"] = links[6 * V:].reshape(3, 4, N, N, N)
            out["piA"] = piA[:3 * V].reshape(3, N, N, N)
            out["piB"] = piA[3 * V:].reshape(3, 3, N, N, N)
        elif links is not None:
            out["links"], out["piA"] = links, piA
        return out

    # -- evolution and observables -----------------------------------------
    def step(self, nsteps: int = 1):
        _check(lib().lattice_step(self.h, ctypes.c_int64(int(nsteps))))

    def energies_noalloc(self) -> dict:
        """lattice_energies_noalloc: the same observables with the library's
        static scratch in place of the workspace's partial sums."""
        o = Obs()
        _check(lib().lattice_energies_noalloc(self.h, ctypes.byref(o)))
        return obs_dict(o, self.nf)

    def energies(self) -> dict:
        o = Obs()
        _check(lib().lattice_energies(self.h, ctypes.byref(o)))
        return obs_dict(o, self.nf)

    def spectrum(self, which: int = 0) -> dict:
        cap = int(np.floor(np.sqrt(3.0) * self.N / 2.0)) + 1
        k, d, s = np.zeros(cap), np.zeros(cap), np.zeros(cap)
        c = np.zeros(cap, dtype=np.int64)
        nb = ctypes.c_int()
        _check(lib().lattice_spectrum(self.h, ctypes.c_int(which), ctypes.c_int(cap), _dp(k), _dp(d), _dp(s),
                                      c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(nb)))
        n = nb.value
        return {"k": k[:n], "delta": d[:n], "S": s[:n], "count": c[:n]}

    def spectrum_logk(self, out, which: int = 1, nk: int = 64):
        """log10 mode-averaged spectrum at nk log-spaced k, written on the device
        into `out` (a float32 CUDA tensor of nk elements, e.g. a row of a
        training set).  Asynchronous on the lattice's stream."""
        import torch
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() < nk or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of at least nk elements")
        _check(lib().lattice_spectrum_logk(self.h, ctypes.c_int(which), ctypes.c_int(nk),
                                           ctypes.c_void_p(out.data_ptr())))

    def pass_timer(self, max_launches: int):
        """Time the next max_launches fused-pass kernels on the device."""
        _check(lib().lattice_pass_timer(self.h, ctypes.c_int32(int(max_launches))))

    def pass_timer_read(self):
        """(summed kernel milliseconds, number of timed launches)."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().lattice_pass_timer_read(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def tiling(self):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().lattice_get_tiling(self.h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_tiling(self, tz, by, ry, xc):
        _check(lib().lattice_set_tiling(self.h, tz, by, ry, xc))

    def close(self):
        if self.h and not self._borrowed:
            lib().lattice_destroy(self.h)
        self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """An ensemble of independent scalar lattices stepped together (one batched
    kernel per pass, whole step calls replayed from a HIP graph).  cfgs: list of
    workload dicts sharing nf, integrator, precision and dt."""

    def __init__(self, cfgs, device: str = "cuda:0", stream=None, ws_fill=None):
        """ws_fill: as for Lattice, a byte written over the workspace first."""
        import torch

        self.cfgs = [dict(c) for c in cfgs]
        n = len(cfgs)
        P = (Params * n)(*[params(c) for c in cfgs])
        self._P = P
        nb = ctypes.c_size_t()
        _check(lib().lattice_batch_workspace_size(P, ctypes.c_int(n), ctypes.byref(nb)))
        self.device = torch.device(device)
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        if ws_fill is not None:
            self.ws.fill_(int(ws_fill))
        base = self.ws.data_ptr()
        off = (-base) % 256
        # graph capture needs a created (non-default) stream; default priority
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        torch.cuda.synchronize(self.device)
        self.h = ctypes.c_void_p()
        _check(lib().lattice_batch_init(P, ctypes.c_int(n), ctypes.c_void_p(base + off), ctypes.c_size_t(nb.value),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.h)))
        self.nruns = n
        self.runs = []
        for r in range(n):
            hr = ctypes.c_void_p()
            _check(lib().lattice_batch_run(self.h, ctypes.c_int(r), ctypes.byref(hr)))
            self.runs.append(Lattice(cfgs[r], _handle=hr, _owner=self))

    def step(self, nsteps: int = 1):
        _check(lib().lattice_batch_step(self.h, ctypes.c_int64(int(nsteps))))

    def energies(self) -> list:
        out = (Obs * self.nruns)()
        _check(lib().lattice_batch_energies(self.h, out))
        return [obs_dict(out[r], self.runs[r].nf) for r in range(self.nruns)]

    def synchronize(self):
        self.stream.synchronize()

    def tiling(self):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().lattice_batch_get_tiling(self.h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_tiling(self, tz, by, ry, xc):
        _check(lib().lattice_batch_set_tiling(self.h, tz, by, ry, xc))

    def use_graph(self, on: bool):
        _check(lib().lattice_batch_use_graph(self.h, 1 if on else 0))

    def close(self):
        if self.h:
            for r in self.runs:
                r.h = ctypes.c_void_p()
            lib().lattice_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
