"""Write the oracle's observables for the full-size parity windows.

Runs the FP64 oracle (OpenMP build) on the benchmarked workloads and stores
its volume observables at checkpoints, so that the GPU tests can compare a
long full-size run without re-running the oracle for minutes.  Only the
oracle is called here.  Each file also records the observables at step 5,
which the GPU tests recompute with the live oracle to show the stored run
still matches it.

    python tests/golden/make_full_size.py [case ...]

Cases (each a file full_size_<case>.json next to this script):
  scalar2_256_vv2_q100    two fields, 256^3, VV2, q = 100, 1000 steps
  scalar2_256_vv2_q1000   the same at q = 1000
  scalar2_256_vv4_q1000   VV4 at q = 1000, 300 steps
  u1higgs_192_lf2         compact U(1), 192^3, staggered leapfrog, 1000 steps
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2006_15122_amd import synth  # noqa: E402

CASES = {
    "scalar2_256_vv2_q100": (lambda: synth.config2(q=100.0, integrator="vv2"), 1000),
    "scalar2_256_vv2_q1000": (lambda: synth.config2(q=1000.0, integrator="vv2"), 1000),
    "scalar2_256_vv4_q1000": (lambda: synth.config2(q=1000.0, integrator="vv4"), 300),
    "u1higgs_192_lf2": (lambda: synth.config3(), 1000),
}
# checkpoints besides every 100 steps: the first 100 steps of the U(1) run
# every 20 (the stretch in which an FP32 run can still follow the FP64 one)
EXTRA = {"u1higgs_192_lf2": [20, 40, 60, 80]}
NSAMPLE = 512


def _clean(o):
    return {k: float(v) for k, v in o.items() if isinstance(v, (float, int, np.floating))}


def _sample_idx(N, ncomp, seed):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, ncomp, NSAMPLE).tolist()] + rng.integers(0, N, (3, NSAMPLE)).tolist()


def run_scalar(name, cfg, nsteps):
    st = oracle.vacuum_ic(cfg)
    m = oracle.scalar_model(cfg)
    phi, pi = st["phi"].copy(), st["pi"].copy()
    a, b = st["a"], st["b"]
    integ, h = cfg["integrator"], cfg["dt"]
    cps = [{"step": 0, "obs": _clean(oracle.sync_observe(m, phi, pi, a, b))}]
    done = 0
    for target in [5] + EXTRA.get(name, []) + list(range(100, nsteps + 1, 100)):
        a, b = oracle.vv_steps(m, phi, pi, a, b, h, integ, target - done, omp=True)
        done = target
        cps.append({"step": done, "obs": _clean(oracle.sync_observe(m, phi, pi, a, b))})
        print(name, "step", done, flush=True)
    idx = _sample_idx(cfg["N"], 2, 11)
    t = tuple(np.array(i) for i in idx)
    return {"checkpoints": cps, "sites": {"idx": idx, "phi": phi[t].tolist(), "pi": pi[t].tolist()}}


def run_u1(name, cfg, nsteps):
    st = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    h = cfg["dt"]
    cps = [{"step": 0, "obs": _clean(oracle.u1_sync_observe(m, st))}]
    oracle.u1_lf_startup(m, st, h)
    done = 0
    for target in [5] + EXTRA.get(name, []) + list(range(100, nsteps + 1, 100)):
        oracle.u1_lf_steps(m, st, h, target - done, omp=True)
        done = target
        cps.append({"step": done, "obs": _clean(oracle.u1_lf_observe(m, st, h))})
        print(name, "step", done, flush=True)
    return {"checkpoints": cps}


def main(names):
    for name in names:
        make, nsteps = CASES[name]
        cfg = make()
        t0 = time.time()
        out = run_u1(name, cfg, nsteps) if cfg["model"] == "u1" else run_scalar(name, cfg, nsteps)
        out.update(case=name, config=cfg, nsteps=nsteps, generator="tests/golden/make_full_size.py",
                   oracle_threads=int(oracle.lib(True).orc_num_threads()), seconds=time.time() - t0)
        with open(os.path.join(HERE, f"full_size_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "written, %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
