"""Benchmark of the lattice hot path on one MI355X.

A step is one full velocity-Verlet (VV2) time step of the two-field model
V = phi^4/4 + q phi^2 chi^2/2 on a 256^3 lattice (FP32 fields and momenta,
FP64 volume averages, self-consistent expansion): drift, stencil kick,
energy reductions and scale-factor update, all in the fused HIP pass.
Inputs are the seeded vacuum initial conditions built on the device.

Prints one JSON line.  value = lattice site-updates per second.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
# (tz, by, ry) shapes the library's autotuner times for FP32 two-field lattices
TUNER_SHAPES = ((64, 4, 2), (64, 8, 2), (32, 8, 2), (128, 8, 2), (256, 4, 2), (128, 4, 2),
                (128, 16, 1), (256, 8, 1), (512, 4, 1))
BYTES_PER_SITE_VV2_NF2_FP32 = 32  # read phi, chi, pi_phi, pi_chi; write the same (FP32)


def _pass_kernel_name(tile) -> str:
    """The FP32 two-field stepping kernel a tile runs: full-row tiles (ry = 1,
    tz = N, four sites per lane) or the general tile."""
    tz, by, ry = tile[:3]
    if ry == 1:
        return "scalar_rows_kernel<float, 4, 2, %d, %d>" % (tz // 4, by)
    return "scalar_pass_kernel<float, 2, false, %d, %d, %d>" % (tz, by, ry)


def _kernel_hash() -> str:
    """Hash of the scalar pass's sources with comments and blank lines left
    out, so that a change to the code, not to its comments, marks the stored
    traffic counters as stale."""
    h = hashlib.sha256()
    for f in ("scalar.hip", "scalar_tile.hpp", "scalar_rows.hpp", "common.hpp"):
        for line in open(os.path.join(ROOT, "paper_2006_15122_amd", "csrc", f)):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _traffic(per_launch_sites: int, tile):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    counts, if they were taken on the current kernel source for this tile;
    else None."""
    p = os.path.join(ROOT, "profiles", "scalar_pass_256_vv2_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != _kernel_hash() or d.get("sites") != per_launch_sites:
        return None
    per = d.get("bytes_per_launch")
    if not isinstance(per, dict):
        return None
    return per.get(",".join(str(v) for v in tile))


def time_lattice(cfg: dict, steps: int, warmup: int, passes: int = 0, tile=None):
    """Time `steps` steps on the lattice's stream (HIP events around the whole
    region).  With passes > 0 a second region of the same `steps` steps
    follows in which the first `passes` fused-pass kernels carry their own
    device start/stop timestamps (hipExtLaunchKernel events, which add a few
    microseconds between launches, so the step time is taken from the first
    region); returns their mean duration as kernel_ms."""
    import torch

    from paper_2006_15122_amd.lattice import Lattice

    lat = Lattice(cfg, device="cuda:0")
    if tile:
        lat.set_tiling(*tile)
    stream = lat.stream
    lat.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    kernel_ms = None
    if passes:
        lat.pass_timer(passes)
        lat.step(steps)
        torch.cuda.synchronize()
        kt, kn = lat.pass_timer_read()
        kernel_ms = kt / kn if kn else None
        lat.pass_timer(0)
    obs = lat.energies()
    tile = lat.tiling()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return ms, wall, obs, tile, kernel_ms


def time_batch(steps: int) -> dict:
    """96 two-field VV2 runs (32 each of 32^3, 64^3, 96^3, q log-uniform in
    [10, 1e4]): one batched kernel per pass replayed from a HIP graph, against
    the same runs stepped one after another with the single-lattice kernels."""
    import torch

    from paper_2006_15122_amd import synth
    from paper_2006_15122_amd.lattice import Batch

    runs = synth.config4_runs()
    B = Batch(runs)
    sites = sum(c["N"] ** 3 for c in runs)
    B.step(steps)                      # captures the graph
    B.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(B.stream)
    B.step(steps)                      # replay
    e1.record(B.stream)
    B.synchronize()
    ms_b = e0.elapsed_time(e1)
    seq_steps = steps                  # the same steps per run as the batched leg
    with torch.cuda.stream(B.stream):
        for r in B.runs:               # warm the single-lattice kernels
            r.step(1)
        B.synchronize()
        e0.record(B.stream)
        for r in B.runs:
            r.step(seq_steps)
        e1.record(B.stream)
        B.synchronize()
    ms_s = e0.elapsed_time(e1)
    tile = B.tiling()
    B.close()
    torch.cuda.empty_cache()
    batched = sites * steps / (ms_b / 1e3)
    seq = sites * seq_steps / (ms_s / 1e3)
    return {"runs": len(runs), "sites": sites, "batched_site_updates_per_s": batched,
            "sequential_site_updates_per_s": seq, "batched_over_sequential": batched / seq,
            "batched_hbm_frac": sites * 32 * (steps + 1) / steps * steps / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS,
            "steps_batched": steps, "steps_sequential": seq_steps, "tile": tile}


def time_surrogate(queries: int = 65536, reps: int = 20) -> dict:
    """Inference of the spectrum surrogate (fused matrix-core forward) on a
    batch of (log10 q, eta) queries, timed with HIP events on its stream.
    Throughput does not depend on the weight values; seeded Glorot weights."""
    import numpy as np
    import torch

    from paper_2006_15122_amd import emulator, synth
    from paper_2006_15122_amd.surrogate import Surrogate

    shift, scale, enc_freq = emulator.in_scaling()
    m = Surrogate(max_batch=64, in_shift=shift, in_scale=scale, enc_freq=enc_freq)
    m.set_weights(synth.mlp_init(1))
    rng = np.random.default_rng(5)
    x = torch.from_numpy(np.stack([1.0 + 3.0 * rng.random(queries), 0.5 + 24.5 * rng.random(queries)],
                                  1).astype(np.float32)).cuda()
    y = torch.empty((queries, 64), dtype=torch.float32, device="cuda:0")
    for _ in range(3):
        m.predict(x, y)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(m.stream)
    for _ in range(reps):
        m.predict(x, y)
    e1.record(m.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    macs = 24 * 256 + 256 * 256 * 2 + 256 * 64      # per query (24 features into the first layer)
    tflops = 2.0 * macs * queries / (ms / 1e3) / 1e12
    m.close()
    return {"queries": queries, "ms_per_batch": ms, "queries_per_s": queries / (ms / 1e3),
            "bf16_tflops": tflops, "mfma_frac": tflops / 2500.0, "kernel": "predict_kernel"}


def time_spectrum(N: int = 256, reps: int = 50) -> dict:
    """One power spectrum of a 256^3 FP32 field (Sec. 3.1): the stored FP32
    values through an FP64 3D FFT, shell binning and the log-k interpolation,
    all queued on the lattice's stream and timed there with HIP events."""
    import torch

    from paper_2006_15122_amd import synth
    from paper_2006_15122_amd.lattice import Lattice

    lat = Lattice(dict(synth.config2(q=100.0), N=N), device="cuda:0")
    out = torch.empty(64, dtype=torch.float32, device="cuda:0")
    for _ in range(5):
        lat.spectrum_logk(out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    for _ in range(reps):
        lat.spectrum_logk(out)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    lat.close()
    del lat
    torch.cuda.empty_cache()
    # algorithmic HBM bytes per spectrum of the three line passes (complex
    # FP64): the z pass reads the FP32 field (4) and writes the complex volume
    # (16), the y pass reads and writes it (32), the x pass reads it (16) and
    # bins in LDS (FP64 sums)
    per_site = 4 + 16 + 32 + 16
    return {"N": N, "ms_per_spectrum": ms, "spectra_per_s": 1e3 / ms, "bytes_per_site": per_site,
            "hbm_frac": N ** 3 * per_site / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg: dict, nsteps: int, st_steps: int) -> dict:
    """The FP64 oracle on the host cores: its OpenMP build over nsteps and its
    single-thread build over st_steps of the same workload."""
    import oracle

    st = oracle.vacuum_ic(cfg)
    m = oracle.scalar_model(cfg)
    N = cfg["N"]
    phi, pi = st["phi"].copy(), st["pi"].copy()
    t0 = time.perf_counter()
    oracle.vv_steps(m, phi, pi, st["a"], st["b"], cfg["dt"], cfg["integrator"], nsteps, omp=True)
    dt = time.perf_counter() - t0
    phi, pi = st["phi"], st["pi"]
    t1 = time.perf_counter()
    oracle.vv_steps(m, phi, pi, st["a"], st["b"], cfg["dt"], cfg["integrator"], st_steps, omp=False)
    dt1 = time.perf_counter() - t1
    return {"value": N ** 3 * nsteps / dt, "unit": "site-updates/s", "cores": int(oracle.lib(True).orc_num_threads()),
            "kind": "oracle", "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"FP64 oracle (C, OpenMP over x-planes), {cfg['integrator'].upper()}, {N}^3, two fields, "
                      f"{nsteps} steps from the seeded initial state, {dt:.1f} s",
            "single_thread": {"value": N ** 3 * st_steps / dt1, "unit": "site-updates/s", "cores": 1,
                              "sample": f"the same oracle built without OpenMP, {st_steps} steps, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--cpu-steps-single", type=int, default=8)
    ap.add_argument("--tile", default=None,
                    help="tz,by,ry,xc of the main run instead of the autotuner's choice (for counter runs, "
                         "where profiling overhead can change the tuner's pick)")
    ap.add_argument("--all-tiles", action="store_true",
                    help="before the timed run, step the workload a few times with every tile the autotuner "
                         "considers (a counter run then covers whichever tile the tuner picks)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy, the reference for HBM counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the lattice runs on a single MI355X "
              f"(--gpus {args.gpus} is not supported: no multi-GPU sharding is implemented)",
              file=sys.stderr)
        sys.exit(2)

    from paper_2006_15122_amd import synth

    if args.calibrate_copy:
        import torch

        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cfg = synth.config2(q=100.0, integrator="vv2")
    N = cfg["N"]
    if args.all_tiles:
        from paper_2006_15122_amd.lattice import Lattice
        lat = Lattice(cfg, device="cuda:0")
        from paper_2006_15122_amd.lattice import LatticeError
        for shape in TUNER_SHAPES:
            for xc in (8, 16, 32, 64):
                try:
                    lat.set_tiling(*shape, xc)
                except LatticeError:
                    continue
                lat.step(4)
        lat.close()
        del lat
    # one call of lattice_step(K) issues K fused passes plus one opening half-kick pass
    passes = args.steps + 1
    forced = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    ms, wall, obs, tile, kernel_ms = time_lattice(cfg, args.steps, args.warmup, passes, forced)
    sites = N ** 3
    # the timed region is the pass kernel back to back (one closing finish
    # kernel per lattice_step call): its duration per launch is the region
    # time over the launches, gaps between launches included
    ms_per_pass = ms / passes
    value = sites * args.steps / (ms / 1e3)
    achieved = sites * BYTES_PER_SITE_VV2_NF2_FP32 / (ms_per_pass / 1e3) / 1e9
    out = {
        "metric": "lattice site-updates/s per GPU (two-field VV2, 256^3, FP32 fields / FP64 sums)",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded vacuum fluctuations, device Philox)",
        "config": {"workload": "two-field preheating phi^4/4 + q phi^2 chi^2/2, q=100, N=256^3, kIR=0.6, "
                               "dt=0.005, velocity Verlet, self-consistent expansion",
                   "N": N, "integrator": "vv2", "nfields": 2, "storage": "fp32", "sums": "fp64",
                   "tile": {"tz": tile[0], "by": tile[1], "ry": tile[2], "xc": tile[3]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": _traffic(sites, tile),
                     "kernel": _pass_kernel_name(tile),
                     "ms_per_launch": ms_per_pass, "launches": passes,
                     "kernel_timing": "HIP events around the timed region on the lattice's stream, divided by "
                                      "the pass launches in it (gaps and the one closing finish kernel included)",
                     "ms_per_launch_ext_events": kernel_ms,
                     "ext_events_note": "per-launch hipExtLaunchKernel start/stop events on a second region of "
                                        "the same steps; within a few percent of the region figure",
                     "bytes_per_launch": sites * BYTES_PER_SITE_VV2_NF2_FP32},
        "wall_s": wall,
        "final_obs": {k: obs[k] for k in ("a", "b", "EK", "EG", "EV", "hc")},
    }
    if not args.no_extras:
        extras = {}
        for name, c, st in (("vv4_256", synth.config2(q=100.0, integrator="vv4"), max(args.steps // 4, 10)),
                            ("vv2_512", dict(synth.config2(q=100.0, N=512), omega_over_f=1e-2), max(args.steps // 8, 10))):
            s_per_site = {"vv2": 1, "vv4": 3}[c["integrator"]]
            npass = st * s_per_site + 1
            ms2, _, _, t2, k2 = time_lattice(c, st, 10, npass)
            n3 = c["N"] ** 3
            extras[name] = {"site_updates_per_s": n3 * st / (ms2 / 1e3),
                            "hbm_frac": n3 * 32 / (ms2 / npass / 1e3) / 1e9 / HBM_PEAK_GBS,
                            "ms_per_pass": ms2 / npass, "ms_per_pass_ext_events": k2, "tile": t2, "steps": st}
        # compact U(1) Abelian-Higgs, 192^3, FP32, staggered leapfrog; state per site: phi (2),
        # pi (2), link phases (3), link momenta (3) = 10 FP32, read and written once per step
        c3 = synth.config3()
        st3 = max(args.steps // 10, 10)
        ms3, _, obs3, _, k3 = time_lattice(c3, st3, 5, st3)
        n3 = c3["N"] ** 3
        extras["u1_192_lf2"] = {"site_updates_per_s": n3 * st3 / (ms3 / 1e3),
                                "hbm_frac": n3 * 80 / (ms3 / st3 / 1e3) / 1e9 / HBM_PEAK_GBS,
                                "ms_per_pass": ms3 / st3, "ms_per_pass_ext_events": k3,
                                "bytes_per_site_update": 80, "steps": st3, "gauss": obs3["gauss"]}
        # the same physics with the non-compact gauge field (Sec. 5.2), same 80 B/site
        c3n = synth.config3_noncompact()
        ms4, _, obs4, _, k4 = time_lattice(c3n, st3, 5, st3)
        extras["u1nc_192_lf2"] = {"site_updates_per_s": n3 * st3 / (ms4 / 1e3),
                                  "hbm_frac": n3 * 80 / (ms4 / st3 / 1e3) / 1e9 / HBM_PEAK_GBS,
                                  "ms_per_pass": ms4 / st3, "ms_per_pass_ext_events": k4,
                                  "bytes_per_site_update": 80, "steps": st3, "gauss": obs4["gauss"]}
        # FP64 storage of the headline workload (the paper's implied precision):
        # 64 B per site-update
        c64 = dict(synth.config2(q=100.0, integrator="vv2"), precision="fp64")
        st64 = max(args.steps // 10, 10)
        ms64, _, _, t64, k64 = time_lattice(c64, st64, 10, st64 + 1)
        n64 = c64["N"] ** 3
        extras["vv2_256_fp64"] = {"site_updates_per_s": n64 * st64 / (ms64 / 1e3),
                                  "hbm_frac": n64 * 64 / (ms64 / (st64 + 1) / 1e3) / 1e9 / HBM_PEAK_GBS,
                                  "ms_per_pass": ms64 / (st64 + 1), "ms_per_pass_ext_events": k64, "tile": t64,
                                  "bytes_per_site_update": 64, "steps": st64}
        # SU(2) x U(1) doublet, 128^3, FP32, velocity Verlet: 35 FP32 per site
        # (Phi 4, pi 4, U(1) phases 3, pi_A 3, SU(2) links 12, pi_B 9) read and
        # written once per pass = 280 B per site-update; each pass is a drift,
        # a kick and a finish kernel
        c5 = synth.config_su2u1()
        st5 = max(args.steps // 20, 10)
        ms5, _, obs5, _, k5 = time_lattice(c5, st5, 5, st5 + 1)
        n5 = c5["N"] ** 3
        extras["su2u1_128_vv2"] = {"site_updates_per_s": n5 * st5 / (ms5 / 1e3),
                                   "hbm_frac": n5 * 280 / (ms5 / (st5 + 1) / 1e3) / 1e9 / HBM_PEAK_GBS,
                                   "ms_per_pass": ms5 / (st5 + 1), "ms_per_kick_kernel": k5,
                                   "bytes_per_site_update": 280, "steps": st5, "gauss": obs5["gauss"],
                                   "gauss_B": obs5["gauss_B"]}
        extras["batch_96"] = time_batch(max(args.steps // 10, 20))
        extras["surrogate_predict_65536"] = time_surrogate()
        extras["spectrum_256"] = time_spectrum()
        out["extras"] = extras
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps, args.cpu_steps_single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
