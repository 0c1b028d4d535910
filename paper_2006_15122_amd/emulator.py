"""Spectrum emulator built on the lattice: training data from batched lattice
runs, a surrogate network trained by the library's own kernels, and the plain
lattice as fallback outside the trained domain.

Inputs of the network are (log10 q, eta) of the two-field model
V = phi^4/4 + q phi^2 chi^2/2 in program units (Sec. 8.1.1 preheating
model with p = 4, vacuum initial fluctuations of Sec. 7.1); outputs are the log10
mode-averaged chi spectrum at 64 log-spaced wavenumbers (Sec. 3.1 binning,
see lattice_spectrum_logk).  Every arithmetic step runs in libcosmolat.so;
this module only schedules calls and moves metadata.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import synth
from .lattice import Batch
from .surrogate import N_OUT, Surrogate

NK = N_OUT
CHI = 1            # field selector of chi in lattice_spectrum_logk


def snapshot_inputs(cfgs, nsnap: int, every: int) -> np.ndarray:
    """(log10 q, eta) of every snapshot, run-major."""
    x = np.zeros((len(cfgs) * nsnap, 2), dtype=np.float32)
    for r, c in enumerate(cfgs):
        for s in range(nsnap):
            x[r * nsnap + s] = (math.log10(c["q"]), (s + 1) * every * c["dt"])
    return x


def generate(cfgs, nsnap: int = 50, every: int = 100, group: int = 256, device: str = "cuda:0",
             progress=None):
    """Run the configurations in batched groups, and after every `every` steps
    write each run's chi spectrum targets into row (run * nsnap + snapshot)
    of T on the device.  Returns (X, T) as CUDA tensors and the seconds spent."""
    import torch
    n = len(cfgs)
    X = torch.from_numpy(snapshot_inputs(cfgs, nsnap, every)).to(device)
    T = torch.empty((n * nsnap, NK), dtype=torch.float32, device=device)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for g0 in range(0, n, group):
        sub = cfgs[g0:g0 + group]
        B = Batch(sub, device=device)
        for s in range(nsnap):
            B.step(every)
            for r, run in enumerate(B.runs):
                run.spectrum_logk(T[(g0 + r) * nsnap + s], which=CHI, nk=NK)
        B.synchronize()
        B.close()
        del B
        if progress:
            progress(g0 + len(sub), n, time.perf_counter() - t0)
    torch.cuda.synchronize(device)
    return X, T, time.perf_counter() - t0


def in_scaling(q_range=(10.0, 1e4), eta_range=(0.5, 25.0), q_gain: float = 24.0, t_gain: float = 6.0,
               enc: float = 1.0):
    """Input normalisation and encoding: the trained domain maps to
    [-q_gain, q_gain] in log10 q and [-t_gain, t_gain] in eta, and the base
    angular frequency of each input's Fourier features is enc pi / gain, so
    that the lowest octave spans half a period over the domain (enc = 1) and
    the highest 2^(octaves-1) times that.  Returns (shift, scale, enc_freq)."""
    lq = (math.log10(q_range[0]), math.log10(q_range[1]))
    shift = (0.5 * (lq[0] + lq[1]), 0.5 * (eta_range[0] + eta_range[1]))
    scale = (2.0 * q_gain / (lq[1] - lq[0]), 2.0 * t_gain / (eta_range[1] - eta_range[0]))
    enc_freq = (enc * math.pi / q_gain, enc * math.pi / t_gain)
    return shift, scale, enc_freq


# Training recipe chosen on a validation split of the training runs: 200 of
# the 2000, recipes of GRID trained on the other 1800, lowest validation MSE
# (select(); `python -m paper_2006_15122_amd.emulator --select`).
DEFAULTS = dict(epochs=5000, lr0=2e-3, enc=0.5)


def train(X, T, epochs: int = DEFAULTS["epochs"], lr0: float = DEFAULTS["lr0"], lr_min: float = 2e-5,
          max_batch: int = 2048, seed: int = 7, q_range=(10.0, 1e4), eta_range=(0.5, 25.0), q_gain: float = 24.0,
          t_gain: float = 6.0, enc: float = DEFAULTS["enc"], device: str = "cuda:0", progress=None,
          progress_every: int = 500):
    """Fit a fresh surrogate to (X, T): output scaling from the targets,
    Glorot initial weights from a seeded generator, Adam with a cosine
    learning-rate decay, a fresh random order of the rows every epoch (one
    permutation buffer, so the library replays its captured epoch)."""
    import torch
    shift, scale, enc_freq = in_scaling(q_range, eta_range, q_gain, t_gain, enc)
    m = Surrogate(device=device, max_batch=max_batch, in_shift=shift, in_scale=scale, enc_freq=enc_freq)
    m.fit_output_scale(T)
    m.set_weights(synth.mlp_init(seed, bias_scale=0.0))
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    hist = []
    perm = torch.empty(n, dtype=torch.int32, device=device)   # one buffer: the captured epoch is replayed
    t0 = time.perf_counter()
    for ep in range(epochs):
        lr = lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * ep / max(1, epochs - 1)))
        perm.copy_(torch.from_numpy(rng.permutation(n).astype(np.int32)))
        loss = m.train_epoch(X, T, perm, lr)
        hist.append(loss)
        if progress and (ep % progress_every == 0 or ep == epochs - 1):
            progress(ep, loss, time.perf_counter() - t0)
    return m, hist, time.perf_counter() - t0


def score(pred, lin, nseeds: int, scatter_max: float = 0.02) -> dict:
    """Relative errors |10^pred - ref| / ref of log10 predictions pred
    (nq, nsnap, NK) against the seed mean ref of the lattice spectra lin
    (nq, nseeds, nsnap, NK, linear).  A point is scored when the scatter of
    the seeds (their standard deviation) is below scatter_max of the mean; the
    suffix _sem marks the looser rule "standard error of the mean below
    scatter_max"."""
    ref = lin.mean(axis=1)
    sd = lin.std(axis=1, ddof=1)
    ok = sd < scatter_max * ref
    ok_sem = sd / math.sqrt(nseeds) < scatter_max * ref
    err = np.abs(10.0 ** pred - ref) / ref
    out = {"err": err, "ok": ok, "ref": ref, "pred": pred}
    for suf, mask in (("", ok), ("_sem", ok_sem)):
        e = err[mask]
        out.update({
            "scored_fraction" + suf: float(mask.mean()),
            "n_scored" + suf: int(mask.sum()),
            "mean_rel_err" + suf: float(e.mean()) if e.size else float("nan"),
            "median_rel_err" + suf: float(np.median(e)) if e.size else float("nan"),
            "p95_rel_err" + suf: float(np.quantile(e, 0.95)) if e.size else float("nan"),
            "max_rel_err" + suf: float(e.max()) if e.size else float("nan"),
        })
    return out


def score_heldout(model: Surrogate, cfgs, nseeds: int, nsnap: int = 50, every: int = 100, scatter_max: float = 0.02,
          device: str = "cuda:0", T=None):
    """Compare the surrogate with the seed mean of plain lattice runs.

    cfgs are grouped by q (nseeds consecutive runs each).  For every q,
    snapshot and wavenumber the reference is the mean over seeds of the
    lattice spectrum 10^t (see score).  Returns the relative errors and
    summary statistics, and the lattice seconds spent."""
    import torch
    if T is None:
        X, T, secs = generate(cfgs, nsnap=nsnap, every=every, device=device)
    else:
        secs = 0.0
    nq = len(cfgs) // nseeds
    t = T.cpu().numpy().astype(np.float64).reshape(nq, nseeds, nsnap, NK)
    xq = snapshot_inputs(cfgs[::nseeds], nsnap, every)
    pred = model.predict(torch.from_numpy(xq).to(device)).cpu().numpy().astype(np.float64)
    out = score(pred.reshape(nq, nsnap, NK), 10.0 ** t, nseeds, scatter_max)
    out["lattice_seconds"] = secs
    return out


def interpolate_in_q(train_cfgs, T_train, query_q, nsnap: int) -> np.ndarray:
    """The plain baseline: for each query q, the log10 spectra of the two
    training runs nearest in log10 q (one seed each), interpolated linearly
    in log10 q per snapshot and wavenumber (the nearest run at the ends).
    T_train: (nruns * nsnap, NK) run-major.  Returns (nq, nsnap, NK)."""
    lq = np.log10(np.array([c["q"] for c in train_cfgs], dtype=np.float64))
    order = np.argsort(lq)
    lqs = lq[order]
    Tt = np.asarray(T_train, dtype=np.float64).reshape(len(train_cfgs), nsnap, -1)[order]
    out = np.zeros((len(query_q), nsnap, Tt.shape[2]))
    for i, q in enumerate(query_q):
        x = math.log10(q)
        j = int(np.searchsorted(lqs, x))
        if j <= 0:
            out[i] = Tt[0]
        elif j >= len(lqs):
            out[i] = Tt[-1]
        else:
            w = (x - lqs[j - 1]) / (lqs[j] - lqs[j - 1])
            out[i] = (1.0 - w) * Tt[j - 1] + w * Tt[j]
    return out


def validation_split(nruns: int, nval: int, seed: int = 99) -> np.ndarray:
    """Boolean mask of nval validation runs drawn from nruns training runs."""
    rng = np.random.default_rng(seed)
    mask = np.zeros(nruns, dtype=bool)
    mask[rng.choice(nruns, nval, replace=False)] = True
    return mask


def validation_error(model: Surrogate, X, T, rows) -> tuple:
    """(normalised mean squared error, mean relative error of 10^y) of the
    model on rows of (X, T): one lattice seed per row, so both include the
    seed scatter, which is the same for every model compared."""
    import torch
    idx = torch.from_numpy(np.asarray(rows, dtype=np.int64)).to(X.device)
    y = model.predict(X.index_select(0, idx).contiguous()).double()
    t = T.index_select(0, idx).double()
    sc = torch.tensor(model.p.out_scale[:], dtype=torch.float64, device=X.device)
    mse = float((((y - t) * sc) ** 2).mean())
    rel = float(((10.0 ** y - 10.0 ** t).abs() / 10.0 ** t).mean())
    return mse, rel


GRID = [dict(epochs=e, lr0=lr, enc=enc) for e in (5000, 20000) for lr in (2e-3,) for enc in (0.5, 1.0, 2.0)]


def select(X, T, nruns: int, nsnap: int, nval: int = 200, grid=GRID, device: str = "cuda:0", progress=None):
    """Train each recipe of the grid on the training runs outside a
    validation split and return (best recipe by validation MSE, table)."""
    import torch
    val = validation_split(nruns, nval)
    rows_tr = np.nonzero(np.repeat(~val, nsnap))[0]
    rows_va = np.nonzero(np.repeat(val, nsnap))[0]
    it = torch.from_numpy(rows_tr.astype(np.int64)).to(X.device)
    Xt, Tt = X.index_select(0, it).contiguous(), T.index_select(0, it).contiguous()
    table = []
    for rec in grid:
        m, hist, secs = train(Xt, Tt, device=device, **rec)
        mse, rel = validation_error(m, X, T, rows_va)
        table.append(dict(rec, val_mse=mse, val_rel=rel, train_loss=hist[-1], seconds=secs))
        if progress:
            progress(table[-1])
        del m
    best = min(table, key=lambda r: r["val_mse"])
    return {k: best[k] for k in ("epochs", "lr0", "enc")}, table


class SpectrumEmulator:
    """Queries (q, eta) -> log10 chi spectrum at NK wavenumbers: the trained
    network inside its domain, a fresh lattice run outside it."""

    def __init__(self, model: Surrogate, q_range=(10.0, 1e4), eta_range=(0.5, 25.0), N: int = 64,
                 every: int = 100, device: str = "cuda:0", fallback_seed: int = 90000):
        self.model = model
        self.q_range, self.eta_range = q_range, eta_range
        self.N, self.every, self.device = N, every, device
        self.fallback_seed = fallback_seed
        self.dt = synth.config2(N=N)["dt"]

    def in_domain(self, q: float, eta: float) -> bool:
        return (self.q_range[0] <= q <= self.q_range[1]) and (self.eta_range[0] <= eta <= self.eta_range[1])

    def lattice(self, q: float, eta: float, seed: int) -> np.ndarray:
        """Plain lattice answer: one run to the step nearest eta."""
        import torch
        c = synth.config2(q=float(q), integrator="vv2", N=self.N, seed=seed)
        steps = max(0, int(round(eta / c["dt"])))
        out = torch.empty(NK, dtype=torch.float32, device=self.device)
        torch.cuda.synchronize(self.device)
        B = Batch([c], device=self.device)
        B.step(steps)
        B.runs[0].spectrum_logk(out, which=CHI, nk=NK)
        B.synchronize()
        B.close()
        return out.cpu().numpy()

    def query(self, q, eta):
        """Arrays of q and eta -> (values [n][NK], source: 1 surrogate, 0 lattice)."""
        import torch
        q = np.atleast_1d(np.asarray(q, dtype=np.float64))
        eta = np.atleast_1d(np.asarray(eta, dtype=np.float64))
        inside = np.array([self.in_domain(a, b) for a, b in zip(q, eta)])
        out = np.zeros((len(q), NK), dtype=np.float32)
        if inside.any():
            x = np.stack([np.log10(q[inside]), eta[inside]], 1).astype(np.float32)
            out[inside] = self.model.predict(torch.from_numpy(x).to(self.device)).cpu().numpy()
        for i in np.nonzero(~inside)[0]:
            out[i] = self.lattice(q[i], eta[i], self.fallback_seed + int(i))
        return out, inside.astype(np.int32)


def main(argv=None):
    """Generate training spectra with the batched lattice, train the
    surrogate, score it on held-out q against seed-averaged lattice runs and
    time both; prints progress lines and one JSON summary line."""
    import argparse
    import json

    import torch

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--train-runs", type=int, default=2000)
    ap.add_argument("--heldout-q", type=int, default=64)
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--N", type=int, default=64)
    ap.add_argument("--nsnap", type=int, default=50)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=DEFAULTS["epochs"])
    ap.add_argument("--lr", type=float, default=DEFAULTS["lr0"])
    ap.add_argument("--enc", type=float, default=DEFAULTS["enc"])
    ap.add_argument("--select", action="store_true",
                    help="first choose epochs, learning rate and encoding frequency on a validation split of "
                         "the training runs (GRID), then train on all of them with the best recipe")
    ap.add_argument("--val-runs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--group", type=int, default=256)
    ap.add_argument("--queries", type=int, default=65536)
    ap.add_argument("--json", default=None, help="also write the summary here")
    ap.add_argument("--save-data", default=None, help="write the training and held-out spectra (npz) here")
    a = ap.parse_args(argv)
    dev = "cuda:0"
    nsteps = a.nsnap * a.every

    def say(*x):
        print(*x, flush=True)

    tr = synth.config5_train_runs(a.train_runs, N=a.N, nsteps=nsteps)
    X, T, tgen = generate(tr, a.nsnap, a.every, a.group, dev,
                          progress=lambda d, n, s: say(f"train data: {d}/{n} runs, {s:.1f} s"))
    site_updates = float(a.train_runs) * a.N ** 3 * nsteps
    say(f"train data: {X.shape[0]} spectra in {tgen:.1f} s ({site_updates / tgen:.3e} site-updates/s)")
    recipe = dict(epochs=a.epochs, lr0=a.lr, enc=a.enc)
    table = None
    if a.select:
        recipe, table = select(X, T, a.train_runs, a.nsnap, a.val_runs, device=dev,
                               progress=lambda r: say("validation: " + json.dumps(r)))
        say("selected " + json.dumps(recipe))
    m, hist, ttrain = train(X, T, max_batch=a.batch, device=dev, **recipe,
                            progress=lambda e, l, s: say(f"epoch {e}: loss {l:.3e}, {s:.1f} s"))
    say(f"trained {recipe['epochs']} epochs in {ttrain:.1f} s, final loss {hist[-1]:.3e}")
    ho = synth.config5_heldout_runs(a.heldout_q, a.seeds, N=a.N, nsteps=nsteps)
    _, TH, tho = generate(ho, a.nsnap, a.every, a.group, dev,
                          progress=lambda d, n, s: say(f"held-out data: {d}/{n} runs, {s:.1f} s"))
    if a.save_data:
        np.savez_compressed(a.save_data, X=X.cpu().numpy(), T=T.cpu().numpy(),
                            XH=snapshot_inputs(ho, a.nsnap, a.every), TH=TH.cpu().numpy(),
                            nseeds=a.seeds, nsnap=a.nsnap)
    J = score_heldout(m, ho, a.seeds, a.nsnap, a.every, T=TH, device=dev)
    say(f"held-out: scored {J['n_scored']} points ({100 * J['scored_fraction']:.1f}%), mean rel err "
        f"{100 * J['mean_rel_err']:.2f}%, p95 {100 * J['p95_rel_err']:.2f}%")
    # the plain alternative: interpolate the training spectra in log10 q
    nq = len(ho) // a.seeds
    pb = interpolate_in_q(tr, T.cpu().numpy(), [c["q"] for c in ho[::a.seeds]], a.nsnap)
    B = score(pb, 10.0 ** TH.cpu().numpy().astype(np.float64).reshape(nq, a.seeds, a.nsnap, NK), a.seeds)
    say(f"interpolation in log10 q between training runs: mean rel err {100 * B['mean_rel_err']:.2f}% "
        f"(looser gate {100 * B['mean_rel_err_sem']:.2f}%)")
    # inference throughput against the lattice's own rate of producing spectra
    rng = np.random.default_rng(123)
    xq = np.stack([1.0 + 3.0 * rng.random(a.queries), 0.5 + 24.5 * rng.random(a.queries)], 1).astype(np.float32)
    xd = torch.from_numpy(xq).to(dev)
    yd = torch.empty((a.queries, NK), dtype=torch.float32, device=dev)
    for _ in range(3):
        m.predict(xd, yd)
    st = m.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(st)
    for _ in range(reps):
        m.predict(xd, yd)
    e1.record(st)
    e1.synchronize()
    t_inf = e0.elapsed_time(e1) / 1e3 / reps
    lattice_rate = X.shape[0] / tgen          # spectra per second from batched lattice runs
    surrogate_rate = a.queries / t_inf
    out = {
        "train_runs": a.train_runs, "N": a.N, "snapshots": a.nsnap, "samples": int(X.shape[0]),
        "data_seconds": tgen, "data_site_updates_per_s": site_updates / tgen,
        "recipe": recipe, "selection": table, "train_seconds": ttrain, "final_loss": hist[-1],
        "heldout_q": a.heldout_q, "seeds": a.seeds,
        **{k: J[k] for k in J if k.startswith(("scored_fraction", "n_scored", "mean_rel_err", "median_rel_err",
                                                 "p95_rel_err", "max_rel_err"))},
        "interp_mean_rel_err": B["mean_rel_err"], "interp_mean_rel_err_sem": B["mean_rel_err_sem"],
        "interp_median_rel_err": B["median_rel_err"],
        "queries": a.queries, "predict_seconds": t_inf, "surrogate_spectra_per_s": surrogate_rate,
        "lattice_spectra_per_s": lattice_rate, "speedup": surrogate_rate / lattice_rate,
    }
    say(json.dumps(out))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    main()
