"""Hubble-constraint ladder of the velocity-Verlet family on the GPU.

Not collected by pytest (a report).  The paper compares its integrators by the
violation of the Hubble constraint, which falls by orders of magnitude from VV2
to VV10 before machine precision stops it (Sec. 8.2.1).  This runs the
two-field model (FP64 storage, so that round-off does not hide the high
orders) to the same time with each integrator and prints the relative
constraint violation |b^2 - (f*/m_p)^2 a^(2(alpha+1)) rho / 3| / b^2.

    python tests/hc_ladder.py [--N 64] [--eta 20] [--dt 0.005]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2006_15122_amd import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=64)
    ap.add_argument("--eta", type=float, default=20.0)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    from paper_2006_15122_amd.lattice import Lattice

    n = int(round(a.eta / a.dt))
    rows = []
    prev = None
    for integ in ("lf2", "vv2", "vv4", "vv6", "vv8", "vv10"):
        cfg = dict(synth.small(synth.config2(q=100.0, integrator=integ), a.N), precision="fp64", dt=a.dt)
        lat = Lattice(cfg, device="cuda:0")
        t0 = time.perf_counter()
        lat.step(n)
        e = lat.energies()
        secs = time.perf_counter() - t0
        gain = "" if prev is None or integ == "vv2" else f"{prev / e['hc']:.3g}"
        rows.append(f"| {integ.upper()} | {e['hc']:.3e} | {gain} | {secs:.2f} |")
        print(rows[-1], flush=True)
        if integ != "lf2":
            prev = e["hc"]
        lat.close()
    lines = [f"Two fields, q = 100, {a.N}^3, FP64 storage, dt = {a.dt}, eta = {a.eta} ({n} steps):", "",
             "| integrator | Hubble-constraint violation | gain over the previous order | seconds |",
             "|---|---|---|---|"] + rows
    print("\n".join(lines))
    if a.out:
        with open(a.out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
