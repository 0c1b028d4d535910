"""Workspaces filled with NaN before init give the same results as zero-filled
ones: no initial condition, pass, partial sum, finish, spectrum or training
step reads workspace memory it has not written first.  0xFF bytes make every
FP32 and FP64 word a NaN, so one stale read anywhere turns a result into NaN
(or, through a comparison, into a different value)."""
import math

import numpy as np
import pytest

from paper_2006_15122_amd import synth

pytestmark = pytest.mark.gpu

POISON, CLEAN = 0xFF, 0x00

CASES = {
    # 96 is not a multiple of 64, so the FP32 passes take their narrow tiles
    "scalar2_vv2_fp32_96": lambda: synth.small(synth.config2(q=100.0), 96),
    "scalar2_vv4_fp64_64": lambda: dict(synth.small(synth.config2(q=100.0, integrator="vv4"), 64),
                                        precision="fp64"),
    "scalar1_lf2_fp64_32": lambda: synth.config1(),
    "u1_lf2_fp32_96": lambda: synth.config3(N=96),
    "u1_lf2_fp64_32": lambda: dict(synth.config3(N=32), precision="fp64"),
    "u1nc_lf2_fp32_64": lambda: synth.config3_noncompact(N=64),
    "su2u1_vv2_fp32_64": lambda: synth.config_su2u1(N=64),
    "su2u1_vv4_fp64_32": lambda: dict(synth.config_su2u1(N=32, integrator="vv4"), precision="fp64"),
}


def _run(cfg, fill, tiling=None):
    from paper_2006_15122_amd.lattice import Lattice

    lat = Lattice(cfg, device="cuda:0", ws_fill=fill)
    if tiling is not None and tuple(lat.tiling()) != tuple(tiling):
        lat.set_tiling(*tiling)   # the pass tile fixes the order of the FP64 partial sums
    lat.step(6)
    out = dict(tiling=lat.tiling(), obs=lat.energies(), state=lat.get_state(),
               spec=lat.spectrum(0))
    lat.step(3)
    out["obs2"] = lat.energies()
    lat.close()
    return out


def _same_obs(a, b):
    for k, v in a.items():
        if isinstance(v, float) and math.isnan(v):
            assert math.isnan(b[k]), k
        else:
            assert v == b[k], (k, v, b[k])


@pytest.mark.parametrize("name", list(CASES))
def test_nan_filled_workspace_gives_the_zero_filled_results(name):
    cfg = CASES[name]()
    print("case", name, flush=True)
    poisoned = _run(cfg, POISON)
    clean = _run(cfg, CLEAN, tiling=poisoned["tiling"])
    for key in ("obs", "obs2"):
        for k in ("a", "b", "EK", "EG", "EV"):
            assert math.isfinite(poisoned[key][k]), (key, k)
        _same_obs(poisoned[key], clean[key])
    for k, v in poisoned["state"].items():
        if isinstance(v, np.ndarray):
            assert np.all(np.isfinite(v)), k
            assert np.array_equal(v, clean["state"][k]), k
    # the shell sums are FP64 atomics: equal up to the order of the additions
    sp, sc = poisoned["spec"], clean["spec"]
    assert np.all(np.isfinite(sp["delta"]))
    assert np.array_equal(sp["count"], sc["count"])
    assert np.allclose(sp["delta"], sc["delta"], rtol=1e-12, atol=0.0)
    assert np.allclose(sp["k"], sc["k"], rtol=1e-12, atol=0.0)


def test_nan_filled_batch_workspace_gives_the_zero_filled_results():
    from paper_2006_15122_amd.lattice import Batch

    cfgs = synth.config4_runs(nruns=6)
    out = []
    for fill in (POISON, CLEAN):
        B = Batch(cfgs, device="cuda:0", ws_fill=fill)
        if out and tuple(B.tiling()) != tuple(out[0][0]):
            B.set_tiling(*out[0][0])
        B.step(4)   # the first call captures the graph, the second replays it
        B.step(4)
        obs = B.energies()
        states = [r.get_state() for r in B.runs]
        out.append((B.tiling(), obs, states))
        B.close()
    for r in range(len(cfgs)):
        for k in ("a", "b", "EK", "EG", "EV"):
            assert math.isfinite(out[0][1][r][k]), (r, k)
        _same_obs(out[0][1][r], out[1][1][r])
        for k, v in out[0][2][r].items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, out[1][2][r][k]), (r, k)


def test_nan_filled_surrogate_workspace_gives_the_zero_filled_results():
    import torch

    from paper_2006_15122_amd.surrogate import Surrogate, pack, unpack

    rng = np.random.default_rng(50)
    n = 700
    x = np.stack([rng.uniform(1.0, 4.0, n), rng.uniform(0.0, 25.0, n)], 1).astype(np.float32)
    t = (-8.0 + rng.standard_normal((n, 64))).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).cuda()
    w = unpack(pack(synth.mlp_init(51, bias_scale=0.2)))
    out = []
    for fill in (POISON, CLEAN):
        m = Surrogate(max_batch=256, in_shift=(2.5, 12.5), in_scale=(1.0 / 1.5, 1.0 / 12.5),
                      enc_freq=(0.9, 0.4), ws_fill=fill)
        sh, sc = m.fit_output_scale(td)
        m.set_weights(w)
        loss, g = m.loss_grad(xd, td, perm[:256].contiguous())
        losses = [m.train_epoch(xd, td, perm, 1e-3) for _ in range(2)]
        y = m.predict(xd).cpu().numpy()
        out.append((sh, sc, loss, g.cpu().numpy(), losses, m.get_weights(), y))
        m.close()
    p, c = out
    assert np.all(np.isfinite(p[6])) and all(math.isfinite(v) for v in p[4])
    assert np.array_equal(p[0], c[0]) and np.array_equal(p[1], c[1])
    assert p[2] == c[2] and p[4] == c[4]
    for i in (3, 5, 6):
        assert np.array_equal(p[i], c[i]), i
