"""Pins of the FP64 MLP oracle against independent library routines and
finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2006_15122_amd import synth


def test_bf16_round_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -0.0, 3.0e38]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp.bf16_round(x)
    assert np.array_equal(got[np.isfinite(ref)], ref[np.isfinite(ref)])
    assert mlp.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0                 # tie -> even (down)
    assert mlp.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6  # tie -> even (up)
    assert mlp.bf16_round(np.array([1.0 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7


def test_gelu_against_normal_cdf_and_its_derivative():
    from scipy.stats import norm
    x = np.linspace(-6, 6, 2001)
    assert np.max(np.abs(mlp.gelu(x) - x * norm.cdf(x))) < 1e-14
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-9


ENC = (0.8, 0.5)


def _batch(seed, B=16):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (B, 2)), rng.standard_normal((B, 64))


def test_features_are_the_inputs_and_their_octave_harmonics():
    u = np.random.default_rng(0).uniform(-3, 3, (50, 2))
    f = mlp.features(u, ENC)
    assert f.shape == (50, 24) and mlp.SIZES[0] == 24
    assert np.array_equal(f[:, :2], u)
    # pairs are (sin, cos) of one angle: unit circle
    for j in range(2, 24, 2):
        assert np.allclose(f[:, j] ** 2 + f[:, j + 1] ** 2, 1.0, atol=1e-15)
    # each octave doubles the angle of the previous one: double-angle formulas
    for c, (start, K) in enumerate(((2, 6), (14, 5))):
        assert np.allclose(f[:, start], np.sin(ENC[c] * u[:, c]), atol=1e-15)
        for k in range(1, K):
            s0, c0 = f[:, start + 2 * (k - 1)], f[:, start + 2 * (k - 1) + 1]
            assert np.allclose(f[:, start + 2 * k], 2 * s0 * c0, atol=1e-12)
            assert np.allclose(f[:, start + 2 * k + 1], c0 ** 2 - s0 ** 2, atol=1e-12)
    # no frequency: the sines vanish and the cosines are one
    f0 = mlp.features(u, (0.0, 0.0))
    assert np.array_equal(f0[:, 2::2], np.zeros((50, 11))) and np.array_equal(f0[:, 3::2], np.ones((50, 11)))


def test_gradients_against_central_differences():
    p = synth.mlp_init(1)
    for k in p:
        p[k] = p[k] + 0.05 * np.random.default_rng(2).standard_normal(p[k].shape)
    x, t = _batch(3)
    L, g = mlp.loss_and_grads(p, x, t, enc_freq=ENC)
    rng = np.random.default_rng(4)
    for k in p:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            h = 1e-5
            p[k][idx] += h
            Lp, _ = mlp.loss_and_grads(p, x, t, enc_freq=ENC)
            p[k][idx] -= 2 * h
            Lm, _ = mlp.loss_and_grads(p, x, t, enc_freq=ENC)
            p[k][idx] += h
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-7 * max(abs(fd), 1e-3), (k, idx, fd, g[k][idx])


def test_gradients_against_torch_autograd_fp64():
    p = synth.mlp_init(5)
    for k in p:
        p[k] = p[k] + 0.05 * np.random.default_rng(6).standard_normal(p[k].shape)
    x, t = _batch(7, B=32)
    L, g = mlp.loss_and_grads(p, x, t, enc_freq=ENC)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    u = torch.tensor(x)
    cols = [u[:, 0:1], u[:, 1:2]]
    for c, K in ((0, 6), (1, 5)):
        for k in range(K):
            a = (2.0 ** k) * ENC[c] * u[:, c:c + 1]
            cols += [torch.sin(a), torch.cos(a)]
    h = torch.cat(cols, 1)
    for l in range(1, 4):
        h = torch.nn.functional.gelu(h @ tp[f"W{l}"].T + tp[f"b{l}"])
    y = h @ tp["W4"].T + tp["b4"]
    Lt = ((y - torch.tensor(t)) ** 2).mean()
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12 * L
    for k in p:
        assert np.max(np.abs(tp[k].grad.numpy() - g[k])) < 1e-12 * max(np.max(np.abs(g[k])), 1e-30), k


def test_bf16_emulation_changes_little():
    p = synth.mlp_init(8)
    x, t = _batch(9, B=64)
    L0, g0 = mlp.loss_and_grads(p, x, t, bf16=False, enc_freq=ENC)
    L1, g1 = mlp.loss_and_grads(p, x, t, bf16=True, enc_freq=ENC)
    assert abs(L1 - L0) < 2e-2 * L0
    for k in g0:
        assert np.linalg.norm(g1[k] - g0[k]) < 5e-2 * np.linalg.norm(g0[k]) + 1e-12, k


def test_adam_against_torch_optim():
    p = synth.mlp_init(10)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    rng = np.random.default_rng(11)
    for _ in range(5):
        g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
        mlp.adam_step(p, g, state, 1e-3)
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
    for k in p:
        assert np.max(np.abs(tp[k].detach().numpy() - p[k])) < 1e-13, k
