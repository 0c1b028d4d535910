"""Pins of the compact U(1) oracle (Sec. 5.3) against facts the paper and the
mathematics fix: Gauss-law conservation to round-off, lattice gauge
invariance, the photon and charged-scalar dispersion relations, the
homogeneous limit against an independent ODE, and the Hubble constraint with
gauge-field energy (which pins the (alpha-1)(E_K^A + E_G^A) term)."""
import math

import numpy as np
import pytest

import oracle
from paper_2006_15122_amd import synth


def _cfg(N=8, e=0.5, expansion=True, alpha=1.0, omega_over_f=0.5, kIR=0.9, seed=7, lam=1.0, m2=(0.0, 0.0)):
    s = 1.0 / math.sqrt(2.0)
    return dict(model="u1", nf=2, N=N, kIR=kIR, dt=0.01, alpha=alpha, fstar_over_mp=2.0,
                omega_over_f=omega_over_f, m2=m2, lam=lam, q=0.0, e=e, phi0=(s, s), dphi0=(0.0, 0.0),
                expansion=expansion, seed=seed, a0=1.0)


def _copy(st):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}


def test_u1_initial_state_has_no_charge_and_satisfies_gauss():
    cfg = _cfg(N=12)
    st = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    g = oracle.u1_gauss(m, st)
    rho = 2 * m.e / m.wf2 * (st["phi"][0] * st["pi"][1] - st["phi"][1] * st["pi"][0])
    assert abs(rho.sum()) < 1e-12 * np.abs(rho).sum()
    assert np.abs(rho).max() > 1e-3           # the fluctuations do carry local charge
    assert math.sqrt(g[0]) < 1e-12 * math.sqrt(g[2])
    assert np.all(st["links"][:, 0] == 1.0) and np.all(st["links"][:, 1] == 0.0)


@pytest.mark.parametrize("h", [0.01, 0.04])
def test_u1_gauss_law_conserved_to_roundoff_with_expansion(h):
    cfg = _cfg(N=8)
    st = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    oracle.u1_lf_startup(m, st, h)
    a0 = st["a"]
    for _ in range(5):
        oracle.u1_lf_steps(m, st, h, 40)
        o = oracle.u1_lf_observe(m, st, h)
        assert o["gauss"] < 1e-12, o["gauss"]
    assert st["a"] > a0 * 1.01
    # the residual measure is not trivially small: perturbing one link momentum breaks it
    st["piA"][0, 1, 2, 3] += 1e-6
    assert oracle.u1_lf_observe(m, st, h)["gauss"] > 1e-9


def _gauge_transform(st, theta):
    """phi -> e^{i th} phi, pi -> e^{i th} pi, V_i(n) -> e^{i th(n)} V_i(n) e^{-i th(n+i)}."""
    out = _copy(st)
    c, s = np.cos(theta), np.sin(theta)
    for key in ("phi", "pi"):
        re, im = st[key][0], st[key][1]
        out[key] = np.stack([c * re - s * im, s * re + c * im])
    L = st["links"]
    newL = np.empty_like(L)
    for i in range(3):
        d = theta - np.roll(theta, -1, axis=i)     # th(n) - th(n+i)
        cd, sd = np.cos(d), np.sin(d)
        newL[i, 0] = cd * L[i, 0] - sd * L[i, 1]
        newL[i, 1] = sd * L[i, 0] + cd * L[i, 1]
    out["links"] = newL
    return out


def test_u1_lattice_gauge_invariance():
    cfg = _cfg(N=6)
    m = oracle.u1_model(cfg)
    rs = synth.random_u1_state(6, seed=3, amp=0.3, link_angle=1.0, emom=0.2)
    st = dict(rs, a=1.0, b=0.3)
    theta = np.random.default_rng(9).uniform(0, 2 * math.pi, (6, 6, 6))
    st2 = _gauge_transform(st, theta)
    o1, o2 = oracle.u1_sync_observe(m, st), oracle.u1_sync_observe(m, st2)
    for k in ("EK", "EG", "EV", "EK_A", "EG_A"):
        assert abs(o1[k] - o2[k]) < 1e-12 * abs(o1[k])
    h = 0.01
    oracle.u1_lf_startup(m, st, h)
    oracle.u1_lf_startup(m, st2, h)
    oracle.u1_lf_steps(m, st, h, 30)
    oracle.u1_lf_steps(m, st2, h, 30)
    st1t = _gauge_transform(st, theta)
    for key in ("phi", "pi", "links", "piA"):
        assert np.max(np.abs(st1t[key] - st2[key])) < 1e-11, key
    assert abs(st["a"] - st2["a"]) < 1e-13


def test_u1_weak_photon_dispersion():
    N, h, nsteps, eps, mm = 12, 0.02, 80, 1e-4, 2
    cfg = _cfg(N=N, expansion=False, e=0.7, kIR=0.8)
    m = oracle.u1_model(cfg)
    dx = m.dx
    x = np.arange(N)[:, None, None] * np.ones((1, N, N))
    A = eps * np.cos(2 * math.pi * mm * x / N + 0.3)
    links = np.zeros((3, 2, N, N, N))
    links[:, 0] = 1.0
    links[1, 0] = np.cos(m.e * dx * A)
    links[1, 1] = -np.sin(m.e * dx * A)
    st = {"phi": np.zeros((2, N, N, N)), "pi": np.zeros((2, N, N, N)), "links": links,
          "piA": np.zeros((3, N, N, N)), "a": 1.0, "b": 0.0}
    oracle.u1_lf_steps(m, st, h, nsteps)
    w2 = (2.0 * math.sin(math.pi * mm / N) / dx) ** 2
    Lm = np.array([[1 - h * h * w2, h], [-h * w2, 1.0]])
    Af, Pf = np.linalg.matrix_power(Lm, nsteps) @ np.array([1.0, 0.0])
    Ay = -np.arctan2(st["links"][1, 1], st["links"][1, 0]) / (m.e * dx)
    mode = np.cos(2 * math.pi * mm * x / N + 0.3)
    assert np.max(np.abs(Ay - eps * Af * mode)) < 1e-6 * eps
    assert np.max(np.abs(st["piA"][1] - eps * Pf * mode)) < 1e-6 * eps * math.sqrt(w2)
    assert np.max(np.abs(st["piA"][0])) == 0.0 and np.max(np.abs(st["piA"][2])) == 0.0


def test_u1_charged_scalar_dispersion_with_trivial_links():
    N, h, nsteps = 8, 0.03, 60
    cfg = _cfg(N=N, expansion=False, lam=0.0, m2=(0.4, 0.0))
    m = oracle.u1_model(cfg)
    nvec = (1, 3, 2)
    xs = np.arange(N)
    X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
    mode = np.cos(2 * math.pi * (nvec[0] * X + nvec[1] * Y + nvec[2] * Z) / N)
    links = np.zeros((3, 2, N, N, N))
    links[:, 0] = 1.0
    st = {"phi": np.stack([0.3 * mode, np.zeros_like(mode)]), "pi": np.zeros((2, N, N, N)),
          "links": links, "piA": np.zeros((3, N, N, N)), "a": 1.0, "b": 0.0}
    # V = m2 |phi|^2, so d/dphi* gives m2 phi: frequency^2 = m2 + k_lat^2
    w2 = 0.4 + sum((2.0 / m.dx * math.sin(math.pi * n / N)) ** 2 for n in nvec)
    oracle.u1_lf_steps(m, st, h, nsteps)
    Lm = np.array([[1 - h * h * w2, h], [-h * w2, 1.0]])
    A, _ = np.linalg.matrix_power(Lm, nsteps) @ np.array([0.3, 0.0])
    assert np.max(np.abs(st["phi"][0] - A * mode)) < 1e-12
    assert np.max(np.abs(st["piA"])) == 0.0


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_u1_homogeneous_against_complex_field_ode(alpha):
    from scipy.integrate import solve_ivp

    lam, fmp, psi0 = 1.0, 2.0, 0.8
    cfg = dict(_cfg(N=4, alpha=alpha), fstar_over_mp=fmp, lam=lam)
    m = oracle.u1_model(cfg)
    T = 1.0

    # phi = (psi + i psi)/sqrt 2 with psi'' + 3 H psi' + 2 lam psi^3 = 0 (cosmic time),
    # rho = psi'^2 + lam psi^4, H = (f*/m_p) sqrt(rho/3)
    def rhs(t, y):
        p, v, aa, eta = y
        H = fmp * math.sqrt((v * v + lam * p ** 4) / 3.0)
        return [v, -3 * H * v - 2 * lam * p ** 3, aa * H, aa ** (-alpha)]

    ev = lambda t, y: y[3] - T
    ev.terminal = True
    sol = solve_ivp(rhs, [0, 50], [psi0, 0.0, 1.0, 0.0], method="DOP853", rtol=1e-13, atol=1e-14, events=ev)
    p_ode, _, a_ode, _ = sol.y_events[0][0]
    errs = []
    for h in (0.01, 0.005):
        links = np.zeros((3, 2, 4, 4, 4))
        links[:, 0] = 1.0
        c = psi0 / math.sqrt(2.0)
        st = {"phi": np.full((2, 4, 4, 4), c), "pi": np.zeros((2, 4, 4, 4)), "links": links,
              "piA": np.zeros((3, 4, 4, 4)), "a": 1.0, "b": fmp * math.sqrt(lam * psi0 ** 4 / 3.0)}
        oracle.u1_lf_startup(m, st, h)
        oracle.u1_lf_steps(m, st, h, int(round(T / h)))
        errs.append((abs(st["a"] - a_ode), abs(st["phi"][0, 0, 0, 0] * math.sqrt(2.0) - p_ode)))
    for j in range(2):
        assert 3.0 < errs[0][j] / errs[1][j] < 5.0, errs
    assert max(errs[1]) < 1e-4


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_u1_hubble_constraint_with_gauge_energy(alpha):
    # a gauge-dominated state: if the (alpha-1)(E_K^A + E_G^A) term of K_a were wrong the
    # constraint would drift at O(1); with it the residual shrinks as h^2
    cfg = dict(_cfg(N=6, alpha=alpha, omega_over_f=1.0), lam=0.05)
    m = oracle.u1_model(cfg)
    rs = synth.random_u1_state(6, seed=11, amp=0.05, link_angle=1.5, emom=1.0)
    base = dict(rs, a=1.0, b=1.0)
    o = oracle.u1_sync_observe(m, base)
    assert o["EK_A"] + o["EG_A"] > 3 * (o["EK"] + o["EG"] + o["EV"])
    base["b"] = math.sqrt(m.fmp2 / 3.0 * o["rho"])
    hcs = []
    for h in (0.01, 0.005):
        st = _copy(base)
        oracle.u1_lf_startup(m, st, h)
        oracle.u1_lf_steps(m, st, h, int(round(0.6 / h)))
        hcs.append(oracle.u1_lf_observe(m, st, h)["hc"])
    assert hcs[0] < 2e-3 and 2.5 < hcs[0] / hcs[1] < 6.0, hcs


# --------------------------------------------------------------------------
# Compact velocity Verlet and its Yoshida compositions (Sec. 5.3.2, 5.3.3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("integ", ["vv2", "vv4"])
def test_u1_vv_conserves_gauss_and_reverses(integ):
    cfg = _cfg(N=8)
    st = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    h = 0.02
    st0 = _copy(st)
    oracle.u1_vv_steps(m, st, h, integ, 30)
    o = oracle.u1_sync_observe(m, st)
    assert o["gauss"] < 1e-12, o["gauss"]
    assert st["a"] > st0["a"] * 1.005
    # time reversal: flip the momenta and b, evolve, flip back
    for k in ("pi", "piA"):
        st[k] = -st[k]
    st["b"] = -st["b"]
    oracle.u1_vv_steps(m, st, h, integ, 30)
    for k in ("pi", "piA"):
        st[k] = -st[k]
    st["b"] = -st["b"]
    for k in ("phi", "pi", "links", "piA"):
        assert np.max(np.abs(st[k] - st0[k])) < 1e-11 * max(1.0, np.max(np.abs(st0[k]))), k
    assert abs(st["a"] - st0["a"]) < 1e-12 and abs(st["b"] - st0["b"]) < 1e-11


@pytest.mark.parametrize("integ,ratio", [("vv2", 4.0), ("vv4", 16.0)])
def test_u1_vv_convergence_order(integ, ratio):
    cfg = _cfg(N=6, omega_over_f=1.0)
    st0 = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    T = 0.4
    res = []
    for h in (0.04, 0.02, 0.01):
        st = _copy(st0)
        oracle.u1_vv_steps(m, st, h, integ, int(round(T / h)))
        res.append(st)
    for key in ("phi", "piA"):
        e1 = np.max(np.abs(res[0][key] - res[1][key]))
        e2 = np.max(np.abs(res[1][key] - res[2][key]))
        assert 0.8 * ratio < e1 / e2 < 1.25 * ratio, (integ, key, e1 / e2)
    ea1, ea2 = abs(res[0]["a"] - res[1]["a"]), abs(res[1]["a"] - res[2]["a"])
    assert 0.8 * ratio < ea1 / ea2 < 1.25 * ratio


def test_u1_vv_and_leapfrog_agree_to_second_order():
    # two different second-order schemes for the same equations: their
    # difference at fixed time shrinks as h^2
    cfg = _cfg(N=6, omega_over_f=1.0)
    st0 = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    T = 0.4
    diffs = []
    for h in (0.02, 0.01):
        n = int(round(T / h))
        v = _copy(st0)
        oracle.u1_vv_steps(m, v, h, "vv2", n)
        lf = _copy(st0)
        oracle.u1_lf_startup(m, lf, h)
        oracle.u1_lf_steps(m, lf, h, n)
        diffs.append(np.max(np.abs(v["phi"] - lf["phi"])))
    assert 3.2 < diffs[0] / diffs[1] < 5.0, diffs
