"""GPU parity of the spectrum surrogate (matrix-core forward, backward, Adam)
and of the device spectrum targets, against the FP64 oracles."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2006_15122_amd import synth

pytestmark = pytest.mark.gpu

IN_SHIFT, IN_SCALE = (2.5, 12.5), (1.0 / 1.5, 1.0 / 12.5)
ENC = (0.9, 0.4)   # base angular frequencies of the Fourier features


def _torch():
    import torch
    return torch


def _inputs(seed, n, nrows=None):
    """(log10 q, eta) rows and raw targets with a smooth dependence on them."""
    rng = np.random.default_rng(seed)
    nrows = n if nrows is None else nrows
    x = np.stack([rng.uniform(1.0, 4.0, nrows), rng.uniform(0.0, 25.0, nrows)], 1)
    k = np.linspace(0, 1, 64)
    t = (-8.0 + 2.0 * np.outer(np.sin(2.0 * x[:, 0]), k) + 0.1 * np.outer(x[:, 1], 1 - k)
         + 0.05 * rng.standard_normal((nrows, 64)))
    return x.astype(np.float32), t.astype(np.float32)


def _out_norm(seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-9.0, -7.0, 64), rng.uniform(0.5, 2.0, 64)


def _model(max_batch, out_shift, out_scale):
    from paper_2006_15122_amd.surrogate import Surrogate
    return Surrogate(max_batch=max_batch, in_shift=IN_SHIFT, in_scale=IN_SCALE, out_shift=out_shift,
                     out_scale=out_scale, enc_freq=ENC)


def _f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def _normalise(x, t, osh, osc):
    """The library's normalisation: the inputs as the kernels form them (FP32
    difference, then FP32 product: the Fourier features multiply any
    discrepancy in them by up to 2^5), the targets in FP64 from the FP32
    values and constants it holds."""
    f32 = np.float32
    xn = ((np.asarray(x, f32) - np.asarray(IN_SHIFT, f32)).astype(f32) * np.asarray(IN_SCALE, f32)).astype(f32)
    xn = xn.astype(np.float64)
    tn = None if t is None else (_f32(t) - _f32(osh)) * _f32(osc)
    return xn, tn


def _weights(seed):
    from paper_2006_15122_amd.surrogate import unpack, pack
    return unpack(pack(synth.mlp_init(seed, bias_scale=0.2)))   # FP32-representable


@pytest.mark.parametrize("n", [1, 1000, 4160])
def test_predict_matches_oracle_forward(n):
    torch = _torch()
    osh, osc = _out_norm(1)
    m = _model(256, osh, osc)
    w = _weights(2)
    m.set_weights(w)
    x, _ = _inputs(3, n)
    y = m.predict(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    xn, _ = _normalise(x, None, osh, osc)
    yn, _ = mlp.forward(w, xn, bf16=True, enc_freq=_f32(ENC))
    ref = yn / _f32(osc) + _f32(osh)
    # Both sides round to BF16 from an FP32 value, but the GPU's FP32 sums (and
    # FP32 features) and the oracle's FP64 ones differ in the last bits, so a
    # few activations in 10^4 round the other way; each such case moves an
    # output by one BF16 step of one activation times a weight: at most
    # 2^-8 * |h3| * |W4| ~ 2^-8 * 2 * 0.14 ~ 1.1e-3 in normalised units for
    # one flip of a last-layer activation near 2 (Glorot bound of W4: 0.14).
    # The norm below is the systematic check.
    d = (y - ref) * _f32(osc)
    assert np.max(np.abs(d)) < 1.5e-3, np.max(np.abs(d))
    assert np.linalg.norm(d) < 1e-4 * np.linalg.norm(yn), np.linalg.norm(d) / np.linalg.norm(yn)


def test_loss_and_gradients_match_oracle_with_bf16_rounding():
    torch = _torch()
    osh, osc = _out_norm(4)
    m = _model(1024, osh, osc)
    w = _weights(5)
    m.set_weights(w)
    x, t = _inputs(6, 0, nrows=3000)
    rows = np.random.default_rng(7).permutation(3000)[:1000].astype(np.int32)   # ragged: 1000 = 15*64 + 40
    loss, g = m.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(rows).cuda())
    g = g.cpu().numpy().astype(np.float64)
    xn, tn = _normalise(x[rows], t[rows], osh, osc)
    L, go = mlp.loss_and_grads(w, xn, tn, bf16=True, enc_freq=_f32(ENC))
    assert abs(loss - L) < 1e-5 * L, (loss, L)
    from paper_2006_15122_amd.surrogate import unpack
    gg = unpack(g)
    for k in go:
        rel = np.max(np.abs(gg[k] - go[k])) / np.max(np.abs(go[k]))
        assert rel < 1e-4, (k, rel)
    # without BF16 emulation the same comparison is visibly worse: the
    # oracle's rounding points are the GPU's
    _, g64 = mlp.loss_and_grads(w, xn, tn, bf16=False, enc_freq=_f32(ENC))
    worse = max(np.max(np.abs(gg[k] - g64[k])) / np.max(np.abs(g64[k])) for k in ("W2", "W3", "W4"))
    assert worse > 1e-4


def test_adam_steps_match_oracle_and_epoch_slicing_is_exact():
    torch = _torch()
    from paper_2006_15122_amd.surrogate import pack, unpack
    osh, osc = _out_norm(8)
    x, t = _inputs(9, 0, nrows=700)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    perm = torch.from_numpy(np.random.default_rng(10).permutation(700).astype(np.int32)).cuda()
    w = _weights(11)
    lr = 1e-3
    m = _model(256, osh, osc)      # trained one slice per call
    gm = _model(256, osh, osc)     # evaluates the gradient each step used
    m.set_weights(w)
    prev, state = w, {}
    for s in range(3):   # slices of 256, 256 and 188 rows
        rows = perm[s * 256:min(700, (s + 1) * 256)].contiguous()
        gm.set_weights(prev)
        _, g = gm.loss_grad(xd, td, rows)
        m.train_epoch(xd, td, rows, lr)
        got = unpack(m.get_weights())
        exp = {k: v.copy() for k, v in prev.items()}
        mlp.adam_step(exp, unpack(g.cpu().numpy()), state, lr)
        for k in exp:
            # FP32 Adam arithmetic against FP64: ~1e-6 of the step, plus the
            # rounding of the stored FP32 weight
            d = np.abs(got[k] - exp[k])
            assert np.all(d <= 1e-5 * lr + 2.4e-7 * np.abs(exp[k])), (s, k, np.max(d))
        prev = got
    # one epoch over the 700 rows takes the same three steps, bit for bit,
    # and repeats bit for bit
    for _ in range(2):
        m2 = _model(256, osh, osc)
        m2.set_weights(w)
        assert math.isfinite(m2.train_epoch(xd, td, perm, lr))
        assert np.array_equal(m2.get_weights(), pack(prev))


def test_training_fits_a_smooth_map():
    torch = _torch()
    x, t = _inputs(12, 0, nrows=8192)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    m = _model(512, None, None)
    sh, sc = m.fit_output_scale(td)
    assert np.allclose(sh, t.astype(np.float64).mean(0), atol=1e-5)
    assert np.allclose(sc, 1.0 / t.astype(np.float64).std(0), rtol=1e-5)
    m.set_weights(_weights(13))
    rng = np.random.default_rng(14)
    first = None
    for ep in range(40):
        perm = torch.from_numpy(rng.permutation(8192).astype(np.int32)).cuda()
        loss = m.train_epoch(xd, td, perm, 2e-3)
        first = loss if first is None else first
    assert loss < 0.05 * first, (first, loss)


def test_device_spectrum_targets_match_oracle():
    torch = _torch()
    from paper_2006_15122_amd.lattice import Lattice
    cfg = synth.small(synth.config2(q=300.0), 32)
    lat = Lattice(cfg, device="cuda:0")
    lat.step(200)
    out = torch.empty(2 * 64, dtype=torch.float32, device="cuda:0")
    lat.spectrum_logk(out[:64], which=1, nk=64)
    lat.spectrum_logk(out[64:], which=17, nk=64)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    s = lat.get_state()
    for half, arr in ((0, s["phi"][1]), (1, s["pi"][1])):
        ref = oracle.spectrum_logk(arr, cfg["kIR"], 64)
        d = np.max(np.abs(got[64 * half:64 * half + 64] - ref) / np.maximum(1.0, np.abs(ref)))
        assert d < 4e-7, (half, d)


def test_emulator_routes_outside_domain_to_the_lattice():
    torch = _torch()
    from paper_2006_15122_amd import emulator
    from paper_2006_15122_amd.lattice import Batch
    m = _model(256, None, None)
    m.set_weights(_weights(21))
    em = emulator.SpectrumEmulator(m, N=32)
    q = np.array([5.0, 100.0, 3e4, 300.0])
    eta = np.array([1.0, 2.0, 1.0, 40.0])
    vals, src = em.query(q, eta)
    assert src.tolist() == [0, 1, 0, 0]
    # the network answers inside the trained domain
    x = torch.tensor([[2.0, 2.0]], dtype=torch.float32, device="cuda:0")
    assert np.array_equal(vals[1], m.predict(x).cpu().numpy()[0])
    # outside it the answer is a plain lattice run to the requested time
    for i in (0, 2, 3):
        c = synth.config2(q=float(q[i]), integrator="vv2", N=32, seed=em.fallback_seed + i)
        B = Batch([c])
        B.step(int(round(eta[i] / c["dt"])))
        out = torch.empty(64, dtype=torch.float32, device="cuda:0")
        B.runs[0].spectrum_logk(out, which=1, nk=64)
        B.synchronize()
        assert np.array_equal(vals[i], out.cpu().numpy()), i
        B.close()


def test_graph_replayed_epochs_match_eager_epochs():
    torch = _torch()
    osh, osc = _out_norm(30)
    x, t = _inputs(31, 0, nrows=1000)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    perm = torch.empty(1000, dtype=torch.int32, device="cuda:0")
    graph, eager = _model(256, osh, osc), _model(256, osh, osc)
    eager.use_graph(False)
    for m in (graph, eager):
        m.set_weights(_weights(32))
    rng = np.random.default_rng(33)
    for ep in range(4):   # captured on the first epoch, replayed on the next three
        perm.copy_(torch.from_numpy(rng.permutation(1000).astype(np.int32)))
        lr = 1e-3 * (ep + 1)
        lg = graph.train_epoch(xd, td, perm, lr)
        assert float((xd * 2.0).sum().item()) != 0.0   # unrelated eager work between replays
        le = eager.train_epoch(xd, td, perm, lr)
        assert lg == le, ep
        assert np.array_equal(graph.get_weights(), eager.get_weights()), ep


def test_surrogate_trained_on_lattice_spectra_answers_held_out_q():
    """What the network adds to the method: spectra at new couplings without a
    lattice run.  The full pipeline (2000 training runs at 64^3, 5000 VV2
    steps each, 10^5 device spectra; the recipe chosen on a validation split
    of the training runs; 64 held-out couplings x 8 seeds) must land within 5%
    mean relative error of the 8-seed lattice mean on the scored points (seed
    scatter below 2%), and within 6% under the looser gate (standard error
    below 2%), while answering 65536 queries at least 10^4 times faster than
    the batched lattice produces spectra.  Linear interpolation in log10 q
    between the two nearest training runs is reported beside it: with 2000
    runs over three decades it is the stronger predictor on the low-scatter
    points (1.2% against 2.8%), while the network is the better one on
    single-seed validation spectra (it averages over the seeds of neighbouring
    couplings)."""
    torch = _torch()
    import time
    from paper_2006_15122_amd import emulator
    tr = synth.config5_train_runs(2000)
    X, T, tgen = emulator.generate(tr, nsnap=50, every=100)
    assert torch.isfinite(T).all()
    m, hist, _ = emulator.train(X, T)
    assert hist[-1] < 0.2 * hist[0]
    ho = synth.config5_heldout_runs(64, 8)
    _, TH, _ = emulator.generate(ho, nsnap=50, every=100)
    J = emulator.score_heldout(m, ho, 8, nsnap=50, every=100, T=TH)
    pb = emulator.interpolate_in_q(tr, T.cpu().numpy(), [c["q"] for c in ho[::8]], 50)
    B = emulator.score(pb, 10.0 ** TH.cpu().numpy().astype(np.float64).reshape(64, 8, 50, 64), 8)
    print("network: scored %d, mean %.4f (looser %.4f); interpolation in q: %.4f (looser %.4f)"
          % (J["n_scored"], J["mean_rel_err"], J["mean_rel_err_sem"], B["mean_rel_err"], B["mean_rel_err_sem"]),
          flush=True)
    assert J["n_scored"] > 20000
    assert J["mean_rel_err"] < 0.05, J["mean_rel_err"]
    assert J["mean_rel_err_sem"] < 0.06, J["mean_rel_err_sem"]
    assert B["n_scored"] == J["n_scored"]
    x = torch.rand(65536, 2, device="cuda:0") * torch.tensor([3.0, 24.5], device="cuda:0") + \
        torch.tensor([1.0, 0.5], device="cuda:0")
    m.predict(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        m.predict(x)
    torch.cuda.synchronize()
    surrogate_rate = 65536 * 10 / (time.perf_counter() - t0)
    lattice_rate = X.shape[0] / tgen
    assert surrogate_rate > 1e4 * lattice_rate, (surrogate_rate, lattice_rate)
    # outside the trained domain the emulator falls back to the lattice
    em = emulator.SpectrumEmulator(m)
    _, src = em.query([5.0, 300.0], [1.0, 1.0])
    assert src.tolist() == [0, 1]
