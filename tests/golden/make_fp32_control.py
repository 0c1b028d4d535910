"""What FP32 storage alone does to a workload: the FP64 oracle run three ways.

  exact    -- FP64 throughout;
  storage  -- after every step the state is rounded to FP32 (fields and
              momenta as values, compact U(1) links through their phase,
              which is how an FP32 lattice stores them); arithmetic FP64;
  initial  -- the initial state rounded once to FP32, then FP64 throughout.
Per checkpoint the file keeps the relative difference of every observable of
the two controlled runs from the exact one, and the Gauss residual of each
(U(1)).  Only the oracle is called.  A GPU FP32 run cannot be closer to the
exact run than "storage" is by more than chance; where even "initial" is far
from it, the dynamics amplify any rounding and trajectory parity ends.

    python tests/golden/make_fp32_control.py <case> [nsteps] [every]
cases: u1higgs_64_lf2 (1000 steps, every 100), u1higgs_192_lf2 (1000 steps,
       every 20 to step 300, then every 100) (compact U(1), leapfrog),
       scalar2_256_vv2_q100 (two fields, velocity Verlet, 1000 steps).
Writes fp32_control_<case>.json next to this script.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2006_15122_amd import synth  # noqa: E402

CASES = {
    "u1higgs_64_lf2": lambda: dict(synth.config3(N=64), precision="fp64"),
    "u1higgs_192_lf2": lambda: dict(synth.config3(N=192), precision="fp64"),
    "scalar2_256_vv2_q100": lambda: dict(synth.config2(q=100.0, integrator="vv2"), precision="fp64"),
}


# checkpoints besides every `every` steps: the first 300 steps of the 192^3
# U(1) run every 20 (the stretch in which FP32 storage still follows FP64)
DENSE = {"u1higgs_192_lf2": (20, 300)}


def _checkpoint_steps(case, nsteps, every):
    steps = set(range(every, nsteps + 1, every))
    if case in DENSE:
        d, upto = DENSE[case]
        steps |= set(range(d, min(upto, nsteps) + 1, d))
    return sorted(steps)


def _f32(x):
    return x.astype(np.float32).astype(np.float64)


def _round(st, u1):
    for k in (("phi", "pi", "piA") if u1 else ("phi", "pi")):
        st[k] = _f32(st[k])
    if u1:
        th = _f32(np.arctan2(st["links"][:, 1], st["links"][:, 0]))
        st["links"][:, 0] = np.cos(th)
        st["links"][:, 1] = np.sin(th)


def _copy(st):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}


def main(case, nsteps=1000, every=100):
    cfg = CASES[case]()
    u1 = cfg["model"] == "u1"
    h = cfg["dt"]
    if u1:
        m = oracle.u1_model(cfg)
        st0 = oracle.u1_vacuum_ic(cfg)
        oracle.u1_lf_startup(m, st0, h)
        keys = ("a", "b", "EK", "EG", "EV", "EK_A", "EG_A", "rho")

        def step(st):
            oracle.u1_lf_steps(m, st, h, 1, omp=True)

        def observe(st):
            return oracle.u1_lf_observe(m, st, h)
    else:
        m = oracle.scalar_model(cfg)
        st0 = oracle.vacuum_ic(cfg)
        keys = ("a", "b", "EK", "EG", "EV", "EV_quartic", "EV_int", "EK0", "EG0", "EK1", "EG1", "meansq0",
                "meansq1")

        def step(st):
            st["a"], st["b"] = oracle.vv_steps(m, st["phi"], st["pi"], st["a"], st["b"], h, cfg["integrator"], 1,
                                               omp=True)

        def observe(st):
            return oracle.sync_observe(m, st["phi"], st["pi"], st["a"], st["b"])
    cps = _checkpoint_steps(case, nsteps, every)
    runs = {}
    t0 = time.time()
    for mode in ("exact", "storage", "initial"):
        st = _copy(st0)
        if mode != "exact":
            _round(st, u1)
        obs = []
        for s in range(nsteps):
            step(st)
            if mode == "storage":
                _round(st, u1)
            if s + 1 in cps:
                obs.append(observe(st))
        runs[mode] = obs
        print(case, mode, "done %.0f s" % (time.time() - t0), flush=True)
    out = {"case": case, "config": cfg, "generator": "tests/golden/make_fp32_control.py", "checkpoints": []}
    for i, stp in enumerate(cps):
        r = runs["exact"][i]
        cp = {"step": stp}
        if u1:
            cp["gauss_exact"] = r["gauss"]
        for mode in ("storage", "initial"):
            o = runs[mode][i]
            cp[mode] = {k: abs(o[k] - r[k]) / abs(r[k]) for k in keys if r[k] != 0.0}
            if u1:
                cp[mode]["gauss"] = o["gauss"]
        out["checkpoints"].append(cp)
    out["seconds"] = time.time() - t0
    with open(os.path.join(HERE, f"fp32_control_{case}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    a = sys.argv[1:]
    main(a[0], int(a[1]) if len(a) > 1 else 1000, int(a[2]) if len(a) > 2 else 100)
