"""Python binding of include/surrogate.h (argument marshalling only).

The network's forward, backward, loss, Adam and inference all run in the HIP
library libcosmolat.so; this module packs weights, allocates the device
workspace with torch and passes pointers and a HIP stream it creates with
torch (ordered against torch's current stream on entry and exit).
"""
from __future__ import annotations

import ctypes

import numpy as np

from .lattice import _check, lib

N_IN, WIDTH, N_OUT = 2, 256, 64
N_FREQ = (6, 5)                      # octaves of the Fourier encoding of each input
N_FEAT = N_IN + 2 * sum(N_FREQ)      # 24 first-layer inputs
NPARAMS = 154432
SHAPES = (("W1", (WIDTH, N_FEAT)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (N_OUT, WIDTH)), ("b4", (N_OUT,)))

EXPORTS = ["surrogate_workspace_size", "surrogate_init", "surrogate_set_weights", "surrogate_get_weights",
           "surrogate_loss_grad", "surrogate_train_epoch", "surrogate_predict", "surrogate_fit_output_scale",
           "surrogate_use_graph", "surrogate_destroy"]


class SurrParams(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("reserved", ctypes.c_int32), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("in_shift", ctypes.c_float * N_IN),
                ("in_scale", ctypes.c_float * N_IN), ("out_shift", ctypes.c_float * N_OUT),
                ("out_scale", ctypes.c_float * N_OUT), ("enc_freq", ctypes.c_float * N_IN)]


def pack(p: dict) -> np.ndarray:
    """Flat FP32 weight vector in the library's order from a dict of arrays."""
    v = np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1) for k, _ in SHAPES]).astype(np.float32)
    assert v.size == NPARAMS
    return v


def unpack(v: np.ndarray) -> dict:
    out, o = {}, 0
    for k, shp in SHAPES:
        n = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def make_params(max_batch=4096, in_shift=(0.0, 0.0), in_scale=(1.0, 1.0), out_shift=None, out_scale=None,
                beta1=0.9, beta2=0.999, eps=1e-8, enc_freq=(0.0, 0.0)) -> SurrParams:
    p = SurrParams()
    p.max_batch = int(max_batch)
    p.beta1, p.beta2, p.eps = float(beta1), float(beta2), float(eps)
    for c in range(N_IN):
        p.in_shift[c], p.in_scale[c] = float(in_shift[c]), float(in_scale[c])
        p.enc_freq[c] = float(enc_freq[c])
    osh = np.zeros(N_OUT) if out_shift is None else np.asarray(out_shift, dtype=np.float64)
    osc = np.ones(N_OUT) if out_scale is None else np.asarray(out_scale, dtype=np.float64)
    for c in range(N_OUT):
        p.out_shift[c], p.out_scale[c] = float(osh[c]), float(osc[c])
    return p


def workspace_size(p: SurrParams) -> int:
    n = ctypes.c_size_t()
    _check(lib().surrogate_workspace_size(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


def _dev(t, dtype, what):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous {dtype} CUDA tensor")
    return t


class Surrogate:
    """The MLP with its device workspace.  x rows are (log10 q, eta); outputs
    are log10 mode-averaged spectra at 64 log-spaced k."""

    def __init__(self, device="cuda:0", stream=None, ws_fill=None, **kw):
        """ws_fill: a byte written over the whole workspace before
        surrogate_init (0xFF: every FP32 word a NaN); kw: make_params."""
        import torch
        self.p = make_params(**kw)
        self.device = torch.device(device)
        nbytes = workspace_size(self.p)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        if ws_fill is not None:
            self.ws.fill_(int(ws_fill))
        # a created stream (default priority), so that training epochs can be
        # captured and replayed as HIP graphs
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        torch.cuda.synchronize(self.device)
        self.h = ctypes.c_void_p()
        _check(lib().surrogate_init(ctypes.byref(self.p), ctypes.c_void_p(self.ws.data_ptr()),
                                    ctypes.c_size_t(nbytes + 256), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(self.h)))

    def _enter(self):
        """Order the library's stream after work already queued by torch."""
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        import torch
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def use_graph(self, on: bool):
        _check(lib().surrogate_use_graph(self.h, 1 if on else 0))

    @property
    def max_batch(self) -> int:
        return int(self.p.max_batch)

    def set_weights(self, w):
        v = pack(w) if isinstance(w, dict) else np.ascontiguousarray(w, dtype=np.float32)
        if v.size != NPARAMS:
            raise ValueError("weight vector has the wrong size")
        _check(lib().surrogate_set_weights(self.h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_weights(self) -> np.ndarray:
        v = np.zeros(NPARAMS, dtype=np.float32)
        _check(lib().surrogate_get_weights(self.h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return v

    def fit_output_scale(self, t):
        """Set the output normalisation to the mean and standard deviation of
        each column of the training targets t (computed on the device)."""
        import torch
        _dev(t, torch.float32, "t")
        sh = np.zeros(N_OUT)
        sc = np.zeros(N_OUT)
        self._enter()
        _check(lib().surrogate_fit_output_scale(self.h, _ptr(t), ctypes.c_int64(t.shape[0]),
                                                sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        for c in range(N_OUT):
            self.p.out_shift[c], self.p.out_scale[c] = sh[c], sc[c]
        return sh, sc

    def loss_grad(self, x, t, rows=None):
        import torch
        _dev(x, torch.float32, "x")
        _dev(t, torch.float32, "t")
        n = int(rows.numel()) if rows is not None else int(x.shape[0])
        if rows is not None:
            _dev(rows, torch.int32, "rows")
        g = torch.empty(NPARAMS, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._enter()
        _check(lib().surrogate_loss_grad(self.h, _ptr(x), _ptr(t), _ptr(rows), ctypes.c_int32(n), _ptr(g),
                                         ctypes.byref(loss)))
        return loss.value, g

    def train_epoch(self, x, t, perm, lr: float) -> float:
        import torch
        _dev(x, torch.float32, "x")
        _dev(t, torch.float32, "t")
        _dev(perm, torch.int32, "perm")
        m = ctypes.c_double()
        self._enter()
        _check(lib().surrogate_train_epoch(self.h, _ptr(x), _ptr(t), _ptr(perm), ctypes.c_int64(perm.numel()),
                                           ctypes.c_double(lr), ctypes.byref(m)))
        return m.value

    def predict(self, x, out=None):
        import torch
        _dev(x, torch.float32, "x")
        if out is None:
            out = torch.empty((x.shape[0], N_OUT), dtype=torch.float32, device=self.device)
        _dev(out, torch.float32, "out")
        self._enter()
        _check(lib().surrogate_predict(self.h, _ptr(x), ctypes.c_int64(x.shape[0]), _ptr(out)))
        self._leave()
        return out

    def close(self):
        if self.h:
            lib().surrogate_destroy(self.h)
        self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
