"""Pins of the non-compact U(1) oracle (Sec. 5.2) against facts the paper and
the mathematics fix: the exact discrete photon solution of the quadratic
gauge sector (pins the sign and the normalisation of the magnetic kernel and
of the drift), Gauss-law conservation to round-off, lattice gauge invariance
under A_i -> A_i + D+_i chi, second-order energy conservation in flat space,
time reversal, and agreement with the compact formulation at weak field to the
order its expansion predicts (which also pins E_G^A against 1 - cos)."""
import math

import numpy as np
import pytest

import oracle


def _cfg(N=8, e=0.5, expansion=True, alpha=1.0, omega_over_f=0.5, kIR=0.9, seed=7, lam=1.0, m2=(0.0, 0.0),
         model="u1nc"):
    s = 1.0 / math.sqrt(2.0)
    return dict(model=model, nf=2, N=N, kIR=kIR, dt=0.01, alpha=alpha, fstar_over_mp=2.0,
                omega_over_f=omega_over_f, m2=m2, lam=lam, q=0.0, e=e, phi0=(s, s), dphi0=(0.0, 0.0),
                expansion=expansion, seed=seed, a0=1.0)


def _copy(st):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}


def _photon(N, m, eps, mm, compact):
    """A_y = eps cos(2 pi mm x / N + 0.3), everything else zero (phi = 0, so
    no current); for the compact model the link V_y = exp(-i e dx A_y)."""
    x = np.arange(N)[:, None, None] * np.ones((1, N, N))
    mode = np.cos(2 * math.pi * mm * x / N + 0.3)
    if compact:
        links = np.zeros((3, 2, N, N, N))
        links[:, 0] = 1.0
        links[1, 0] = np.cos(m.e * m.dx * eps * mode)
        links[1, 1] = -np.sin(m.e * m.dx * eps * mode)
    else:
        links = np.zeros((3, N, N, N))
        links[1] = eps * mode
    st = {"phi": np.zeros((2, N, N, N)), "pi": np.zeros((2, N, N, N)), "links": links,
          "piA": np.zeros((3, N, N, N)), "a": 1.0, "b": 0.0}
    return st, mode


def _Ay(st, m, compact):
    if compact:
        return -np.arctan2(st["links"][1, 1], st["links"][1, 0]) / (m.e * m.dx)
    return st["links"][1]


def test_noncompact_photon_is_the_exact_discrete_wave():
    """Quadratic gauge sector: a transverse mode obeys A'' = -w^2 A with the
    lattice w^2 = (2 sin(pi m/N)/dx)^2, and velocity Verlet maps (A, piA) by
    the known 2x2 matrix, to round-off, at any amplitude."""
    N, h, nsteps, eps, mm = 12, 0.02, 80, 0.7, 2
    cfg = _cfg(N=N, expansion=False, e=0.7, kIR=0.8)
    m = oracle.u1_model(cfg)
    st, mode = _photon(N, m, eps, mm, compact=False)
    oracle.u1_vv_steps(m, st, h, "vv2", nsteps)
    w2 = (2.0 * math.sin(math.pi * mm / N) / m.dx) ** 2
    M = np.array([[1 - h * h * w2 / 2, h], [-h * w2 * (1 - h * h * w2 / 4), 1 - h * h * w2 / 2]])
    A, P = np.linalg.matrix_power(M, nsteps) @ np.array([eps, 0.0])
    assert np.max(np.abs(st["links"][1] - A * mode)) < 1e-12
    assert np.max(np.abs(st["piA"][1] - P * mode)) < 1e-11
    for i in (0, 2):
        assert np.max(np.abs(st["links"][i])) == 0.0 and np.max(np.abs(st["piA"][i])) == 0.0
    assert np.max(np.abs(st["phi"])) == 0.0
    # the magnetic energy of the mode is the quadratic one: (w*/f*)^2 <F_xy^2> / 2
    o = oracle.u1_sync_observe(m, st)
    F = (np.roll(st["links"][1], -1, axis=0) - st["links"][1]) / m.dx
    assert abs(o["EG_A"] - m.wf2 * np.mean(F * F) / 2.0) < 1e-13 * o["EG_A"]


def test_noncompact_matches_compact_at_weak_field_to_third_order():
    """The compact theory is the non-compact one plus corrections cubic in
    the plaquette angle (sin x = x - x^3/6, 2 atan(u) = 2u - 2u^3/3): the
    relative difference of the evolved fields falls 4x when the amplitude
    halves, and the magnetic energies differ by a relative O(angle^2)."""
    N, h, nsteps, mm = 12, 0.02, 60, 3
    diffs, ediffs = [], []
    for eps in (0.4, 0.2, 0.1):
        out = []
        for compact in (True, False):
            cfg = _cfg(N=N, expansion=False, e=0.9, kIR=0.8, model="u1" if compact else "u1nc")
            m = oracle.u1_model(cfg)
            st, _ = _photon(N, m, eps, mm, compact)
            oracle.u1_vv_steps(m, st, h, "vv2", nsteps)
            out.append((_Ay(st, m, compact), st["piA"][1], oracle.u1_sync_observe(m, st)["EG_A"]))
        diffs.append(np.max(np.abs(out[0][0] - out[1][0])) / eps)
        ediffs.append(abs(out[0][2] - out[1][2]) / out[1][2])
    for d in (diffs, ediffs):
        assert 3.5 < d[0] / d[1] < 4.5 and 3.5 < d[1] / d[2] < 4.5, d
    assert diffs[2] < 1e-3


@pytest.mark.parametrize("scheme", ["lf", "vv2", "vv4"])
def test_noncompact_gauss_law_conserved_with_expansion(scheme):
    cfg = _cfg(N=8)
    st = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    assert st["links"].shape == (3, 8, 8, 8) and m.noncompact == 1
    h = 0.02
    a0 = st["a"]
    if scheme == "lf":
        oracle.u1_lf_startup(m, st, h)
        oracle.u1_lf_steps(m, st, h, 60)
        o = oracle.u1_lf_observe(m, st, h)
    else:
        oracle.u1_vv_steps(m, st, h, scheme, 60 if scheme == "vv2" else 20)
        o = oracle.u1_sync_observe(m, st)
    assert o["gauss"] < 1e-12, o["gauss"]
    assert st["a"] > a0 * 1.005
    assert np.max(np.abs(st["links"])) > 1e-3      # the current did source the gauge field
    st["piA"][0, 1, 2, 3] += 1e-6
    assert oracle.u1_sync_observe(m, st)["gauss"] > 1e-9


def test_noncompact_gauge_invariance():
    """phi -> e^{i th} phi, A_i -> A_i + (th(n+i) - th(n)) / (e dx) leaves the
    energies and the evolution covariant (V_i = exp(-i e dx A_i))."""
    N = 6
    cfg = _cfg(N=N, expansion=True)
    m = oracle.u1_model(cfg)
    st = oracle.u1_vacuum_ic(cfg)
    rng = np.random.default_rng(4)
    st["links"] = rng.uniform(-0.5, 0.5, (3, N, N, N))
    theta = rng.uniform(0, 2 * math.pi, (N, N, N))

    def transform(s):
        out = _copy(s)
        c, sn = np.cos(theta), np.sin(theta)
        for key in ("phi", "pi"):
            re, im = s[key][0], s[key][1]
            out[key] = np.stack([c * re - sn * im, sn * re + c * im])
        out["links"] = np.stack([s["links"][i] + (np.roll(theta, -1, axis=i) - theta) / (m.e * m.dx)
                                 for i in range(3)])
        return out

    st2 = transform(st)
    o1, o2 = oracle.u1_sync_observe(m, st), oracle.u1_sync_observe(m, st2)
    for k in ("EK", "EG", "EV", "EK_A", "EG_A"):
        assert abs(o1[k] - o2[k]) < 1e-12 * abs(o1[k]), k
    h = 0.01
    oracle.u1_vv_steps(m, st, h, "vv2", 20)
    oracle.u1_vv_steps(m, st2, h, "vv2", 20)
    st1t = transform(st)
    for key in ("phi", "pi", "links", "piA"):
        assert np.max(np.abs(st1t[key] - st2[key])) < 1e-10, key
    assert abs(st["a"] - st2["a"]) < 1e-13


def test_noncompact_energy_conserved_to_second_order_in_flat_space():
    """No expansion: the total energy of the symplectic scheme oscillates at
    O(h^2) about a constant; halving h divides the excursion by 4."""
    cfg = _cfg(N=8, expansion=False, omega_over_f=1.0)
    st0 = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    T = 1.2
    exc = []
    for h in (0.04, 0.02):
        st = _copy(st0)
        E = []
        for _ in range(int(round(T / h))):
            oracle.u1_vv_steps(m, st, h, "vv2", 1)
            o = oracle.u1_sync_observe(m, st)
            E.append(o["rho"])
        E = np.array(E)
        exc.append(np.max(np.abs(E - E[0])) / E[0])
    assert exc[0] < 1e-2
    assert 3.0 < exc[0] / exc[1] < 5.0, exc


@pytest.mark.parametrize("integ", ["vv2", "vv4"])
def test_noncompact_vv_reverses(integ):
    cfg = _cfg(N=8)
    st = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    h = 0.02
    oracle.u1_vv_steps(m, st, h, integ, 10)     # start from a state with A != 0
    st0 = _copy(st)
    oracle.u1_vv_steps(m, st, h, integ, 20)
    for k in ("pi", "piA"):
        st[k] = -st[k]
    st["b"] = -st["b"]
    oracle.u1_vv_steps(m, st, h, integ, 20)
    for k in ("pi", "piA"):
        st[k] = -st[k]
    st["b"] = -st["b"]
    for k in ("phi", "pi", "links", "piA"):
        assert np.max(np.abs(st[k] - st0[k])) < 1e-11 * max(1.0, np.max(np.abs(st0[k]))), k
    assert abs(st["a"] - st0["a"]) < 1e-12 and abs(st["b"] - st0["b"]) < 1e-11


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_noncompact_hubble_constraint_gauge_dominated(alpha):
    """A gauge-dominated expanding state: the Hubble constraint stays satisfied
    to O(h^2) only if the drift A' = a^{-(1-alpha)} piA, the magnetic kernel,
    E_G^A and the (alpha-1)(E_K^A + E_G^A) term of K_a are mutually consistent."""
    N = 6
    cfg = dict(_cfg(N=N, alpha=alpha, omega_over_f=1.0), lam=0.05)
    m = oracle.u1_model(cfg)
    rng = np.random.default_rng(11)
    s = 1.0 / math.sqrt(2.0)
    base = {"phi": np.stack([s + 0.05 * rng.standard_normal((N, N, N)), s + 0.05 * rng.standard_normal((N, N, N))]),
            "pi": np.zeros((2, N, N, N)), "links": 1.5 * rng.standard_normal((3, N, N, N)),
            "piA": rng.standard_normal((3, N, N, N)), "a": 1.0, "b": 1.0}
    o = oracle.u1_sync_observe(m, base)
    assert o["EK_A"] + o["EG_A"] > 3 * (o["EK"] + o["EG"] + o["EV"])
    base["b"] = math.sqrt(m.fmp2 / 3.0 * o["rho"])
    hcs = []
    for h in (0.01, 0.005):
        st = _copy(base)
        oracle.u1_vv_steps(m, st, h, "vv2", int(round(0.6 / h)))
        hcs.append(oracle.u1_sync_observe(m, st)["hc"])
    assert st["a"] > 1.1
    assert hcs[0] < 1e-2 and 3.0 < hcs[0] / hcs[1] < 5.0, hcs
