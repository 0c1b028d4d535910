"""GPU checks of batched ensembles: one batched kernel per pass over the
tiles of runs of different sizes, replayed from a HIP graph."""
import numpy as np
import pytest

import oracle
from paper_2006_15122_amd import synth

pytestmark = pytest.mark.gpu


def _runs(sizes=(32, 64, 96, 32, 64, 96), nsteps=100, integ="vv2"):
    out = []
    qs = [30.0, 300.0, 3000.0, 100.0, 1000.0, 10.0]
    for i, N in enumerate(sizes):
        c = synth.config2(q=qs[i % len(qs)], integrator=integ, N=N, seed=4000 + i)
        c["nsteps"] = nsteps
        out.append(c)
    return out


def _rel(a, b):
    return abs(a - b) / abs(b)


def test_batch_matches_individual_runs_and_oracle():
    from paper_2006_15122_amd.lattice import Batch, Lattice

    cfgs = _runs()
    B = Batch(cfgs)
    B.step(120)
    eb = B.energies()
    for r, c in enumerate(cfgs):
        L = Lattice(c)
        L.step(120)
        e = L.energies()
        for k in ("a", "b", "EK", "EG", "EV"):
            assert _rel(eb[r][k], e[k]) < 1e-6, (r, k, eb[r][k], e[k])
        L.close()
    # run 0 against the FP64 oracle from the same device initial state
    c = cfgs[0]
    st = oracle.vacuum_ic(c)
    m = oracle.scalar_model(c)
    a, b = oracle.vv_steps(m, st["phi"], st["pi"], st["a"], st["b"], c["dt"], "vv2", 120)
    o = oracle.sync_observe(m, st["phi"], st["pi"], a, b)
    for k in ("a", "b", "EK", "EG", "EV"):
        assert _rel(eb[0][k], o[k]) < 1e-5, (k, eb[0][k], o[k])
    B.close()


def test_graph_replays_match_eager_launches():
    from paper_2006_15122_amd.lattice import Batch

    cfgs = _runs(sizes=(32, 64, 32, 96))
    G = Batch(cfgs)
    E = Batch(cfgs)
    E.use_graph(False)
    E.set_tiling(*G.tiling())
    for rep in range(4):
        G.step(25)          # captured on the first call, replayed afterwards
        E.step(25)
        eg, ee = G.energies(), E.energies()   # eager work and syncs between replays
        for r in range(len(cfgs)):
            sg = G.runs[r].get_state()
            se = E.runs[r].get_state()
            assert np.array_equal(sg["phi"], se["phi"]), (rep, r)
            assert np.array_equal(sg["pi"], se["pi"]), (rep, r)
            assert sg["a"] == se["a"] and sg["b"] == se["b"]
            assert eg[r]["EK"] == ee[r]["EK"]
    G.close()
    E.close()


def test_batch_vv4_and_run_handles():
    from paper_2006_15122_amd.lattice import Batch

    cfgs = _runs(sizes=(32, 64), integ="vv4")
    B = Batch(cfgs)
    st = oracle.vacuum_ic(cfgs[1])
    B.runs[1].set_state(st["phi"], st["pi"], st["a"], st["b"])
    B.step(40)
    e = B.energies()[1]
    m = oracle.scalar_model(cfgs[1])
    a, b = oracle.vv_steps(m, st["phi"], st["pi"], st["a"], st["b"], cfgs[1]["dt"], "vv4", 40, omp=True)
    o = oracle.sync_observe(m, st["phi"], st["pi"], a, b)
    for k in ("a", "b", "EK", "EG", "EV"):
        assert _rel(e[k], o[k]) < 1e-5, (k, e[k], o[k])
    s = B.runs[1].get_state()
    assert s["step"] == 40
    B.close()


def test_every_batch_tiling_against_oracle():
    """Every compiled batch tile shape and x-chunk that divides all three sizes,
    each run against the FP64 oracle from the same state (6 VV2 steps)."""
    from paper_2006_15122_amd.lattice import Batch

    cfgs = _runs(sizes=(32, 64, 96))
    states = [synth.random_state(c, seed=50 + r, amp=0.2, mom=0.2) for r, c in enumerate(cfgs)]
    ref = []
    for c, st in zip(cfgs, states):
        m = oracle.scalar_model(c)
        phi, pi = st["phi"].copy(), st["pi"].copy()
        a, b = oracle.vv_steps(m, phi, pi, 1.0, 0.3, c["dt"], "vv2", 6, omp=True)
        ref.append(oracle.sync_observe(m, phi, pi, a, b))
    B = Batch(cfgs)
    n = 0
    for (tz, by, ry) in [(32, 8, 2), (32, 4, 4), (32, 8, 4), (64, 4, 2), (64, 4, 4)]:
        for xc in (8, 16, 32):
            try:
                B.set_tiling(tz, by, ry, xc)
            except Exception:
                continue
            for r, st in enumerate(states):
                B.runs[r].set_state(st["phi"], st["pi"], 1.0, 0.3)
            B.step(6)
            for r, e in enumerate(B.energies()):
                for k in ("a", "b", "EK", "EG", "EV"):
                    assert _rel(e[k], ref[r][k]) < 1e-5, (tz, by, ry, xc, r, k, e[k], ref[r][k])
            n += 1
    assert n >= 6
    B.close()


def test_chained_finish_of_each_run_is_its_own():
    # each pass reduces its own run's records of the previous pass (the run's
    # slice of the tile table) and stores the run's state slots; a batch of
    # three runs must therefore give each run the bits of a batch of that run
    # alone on the same tile
    from paper_2006_15122_amd.lattice import Batch

    cfgs = _runs(sizes=(32, 96, 64), integ="vv4")
    B = Batch(cfgs)
    B.step(23)
    B.step(4)
    for r, c in enumerate(cfgs):
        S = Batch([c])
        S.set_tiling(*B.tiling())
        S.step(23)
        S.step(4)
        sb, ss = B.runs[r].get_state(), S.runs[0].get_state()
        assert np.array_equal(sb["phi"], ss["phi"]) and np.array_equal(sb["pi"], ss["pi"]), r
        assert sb["a"] == ss["a"] and sb["b"] == ss["b"] and sb["eta"] == ss["eta"], r
        S.close()
    B.close()
