"""Pins of the SU(2) x U(1) doublet oracle (Sec. 6; initial state Sec. 7.2)
against facts the paper and the mathematics fix: both Gauss laws conserved to
round-off for every integrator with expansion on, invariance under random
lattice SU(2) x U(1) gauge transformations, unitary links, time reversal,
convergence orders, conservation of the total energy in flat space (which
fixes every relative normalisation of kernels and energies), the free
non-Abelian wave, the homogeneous limit against an independent ODE, and two
reductions to the separately pinned U(1) model: the upper doublet component
alone with the SU(2) coupling switched off, and SU(2) links in the sigma_3
subgroup, which act as a U(1) field of charge g/2."""
import math

import numpy as np
import pytest

import oracle


def _cfg(N=6, e=0.3, g=0.5, expansion=True, alpha=1.0, omega_over_f=0.5, kIR=0.9, seed=7, lam=1.0, m2=(0.0, 0.0),
         phi0=(0.5, 0.5, 0.5, 0.5)):
    return dict(model="su2u1", N=N, kIR=kIR, dt=0.01, alpha=alpha, fstar_over_mp=2.0, omega_over_f=omega_over_f,
                m2=m2, lam=lam, e=e, g=g, phi0=phi0, dphi0=(0.0,) * 4, expansion=expansion, seed=seed, a0=1.0)


def _copy(st):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}


def _random_state(N, seed, amp=0.2, link_angle=0.8, emom=0.3):
    """Seeded random doublet state with random U(1) and SU(2) links."""
    rng = np.random.default_rng(seed)
    phi = 0.5 + amp * (rng.random((4, N, N, N)) - 0.5)
    pi = amp * (rng.random((4, N, N, N)) - 0.5)
    th = link_angle * (rng.random((3, N, N, N)) - 0.5)
    links = np.stack([np.cos(th), np.sin(th)], axis=1)
    v = link_angle * (rng.random((3, 3, N, N, N)) - 0.5)
    ang = np.sqrt((v * v).sum(axis=1))
    n = v / np.where(ang > 0, ang, 1.0)[:, None]
    su2 = np.concatenate([np.cos(ang)[:, None], np.sin(ang)[:, None] * n], axis=1)
    assert np.max(np.abs((su2 ** 2).sum(axis=1) - 1.0)) < 1e-14
    piA = emom * (rng.random((3, N, N, N)) - 0.5)
    piB = emom * (rng.random((3, 3, N, N, N)) - 0.5)
    return {"phi": phi, "pi": pi, "links": links, "su2": np.ascontiguousarray(su2), "piA": piA, "piB": piB}


def test_su2_initial_state_has_no_charges_and_satisfies_both_gauss_laws():
    cfg = _cfg(N=10)
    st = oracle.su2_vacuum_ic(cfg)
    m = oracle.su2_model(cfg)
    rA, rB = oracle.su2_charges(cfg, st["phi"], st["pi"])
    assert abs(rA.sum()) < 1e-12 * np.abs(rA).sum() and np.abs(rA).max() > 1e-3
    for c in range(3):
        assert abs(rB[c].sum()) < 1e-12 * np.abs(rB[c]).sum() and np.abs(rB[c]).max() > 1e-3
    o = oracle.su2_sync_observe(m, st)
    assert o["gauss"] < 1e-13 and o["gauss_B"] < 1e-13
    assert o["EG_A"] == 0.0 and o["EG_B"] == 0.0 and o["EK_B"] > 0.0
    assert np.all(st["su2"][:, 0] == 1.0) and np.all(st["su2"][:, 1:] == 0.0)


@pytest.mark.parametrize("integ,h", [("lf2", 0.01), ("lf2", 0.04), ("vv2", 0.02), ("vv4", 0.02)])
def test_su2_gauss_laws_conserved_to_roundoff_with_expansion(integ, h):
    cfg = _cfg(N=6)
    st = oracle.su2_vacuum_ic(cfg)
    m = oracle.su2_model(cfg)
    a0 = st["a"]
    if integ == "lf2":
        oracle.su2_lf_startup(m, st, h)
    for _ in range(3):
        if integ == "lf2":
            oracle.su2_lf_steps(m, st, h, 20)
            o = oracle.su2_lf_observe(m, st, h)
        else:
            oracle.su2_vv_steps(m, st, h, integ, 10)
            o = oracle.su2_sync_observe(m, st)
        assert o["gauss"] < 1e-12 and o["gauss_B"] < 1e-12, (o["gauss"], o["gauss_B"])
    assert st["a"] > a0 * 1.005
    assert o["EG_B"] > 0.0
    # the residuals are not trivially small: one perturbed link momentum breaks each
    st["piB"][1, 2, 1, 2, 3] += 1e-6
    st["piA"][0, 3, 2, 1] += 1e-6
    o = oracle.su2_sync_observe(m, st)
    assert o["gauss"] > 1e-9 and o["gauss_B"] > 1e-9


def _su2_exp(v):
    """exp(i v.sigma) as (c0, c): cos|v| + i sin|v| v/|v| . sigma."""
    ang = np.sqrt((v * v).sum(axis=0))
    n = v / np.where(ang > 0, ang, 1.0)
    return np.concatenate([np.cos(ang)[None], np.sin(ang)[None] * n], axis=0)


def _mat(c):
    """2x2 complex matrices [[c0 + i c3, c2 + i c1], [-c2 + i c1, c0 - i c3]] over the lattice."""
    return np.array([[c[0] + 1j * c[3], c[2] + 1j * c[1]], [-c[2] + 1j * c[1], c[0] - 1j * c[3]]])


def _c_of(M):
    return np.stack([M[0, 0].real, M[0, 1].imag, M[0, 1].real, M[0, 0].imag])


def _mm(A, B):
    return np.einsum("ij...,jk...->ik...", A, B)


def _dag(A):
    return np.conj(np.swapaxes(A, 0, 1))


def _gauge_transform(st, beta, gam):
    """Phi -> e^{i beta} Om Phi, pi likewise, V_i(n) -> e^{i beta(n)} V_i(n) e^{-i beta(n+i)},
    U_i(n) -> Om(n) U_i(n) Om(n+i)^dag, pi_A unchanged, pi_B,i(n) -> Om(n) pi_B,i(n) Om(n)^dag,
    with Om = exp(i gam.sigma)."""
    out = _copy(st)
    Om = _mat(_su2_exp(gam))
    ph = np.exp(1j * beta)
    for key in ("phi", "pi"):
        x = st[key]
        v = np.array([x[0] + 1j * x[1], x[2] + 1j * x[3]])
        w = np.einsum("ij...,j...->i...", Om, v) * ph
        out[key] = np.stack([w[0].real, w[0].imag, w[1].real, w[1].imag])
    L = st["links"]
    newL = np.empty_like(L)
    newU = np.empty_like(st["su2"])
    newB = np.empty_like(st["piB"])
    sig = [np.array([[0, 1], [1, 0]], dtype=complex), np.array([[0, -1j], [1j, 0]]),
           np.array([[1, 0], [0, -1]], dtype=complex)]
    for i in range(3):
        d = beta - np.roll(beta, -1, axis=i)
        V = (L[i, 0] + 1j * L[i, 1]) * np.exp(1j * d)
        newL[i, 0], newL[i, 1] = V.real, V.imag
        Omp = np.roll(Om, -1, axis=2 + i)
        newU[i] = _c_of(_mm(_mm(Om, _mat(st["su2"][i])), _dag(Omp)))
        P = sum(st["piB"][i, a] * sig[a][:, :, None, None, None] / 2 for a in range(3))
        Q = _mm(_mm(Om, P), _dag(Om))
        for a in range(3):
            newB[i, a] = np.einsum("ij...,ji...->...", sig[a][:, :, None, None, None] * np.ones_like(Q), Q).real
    out["links"], out["su2"], out["piB"] = newL, newU, newB
    return out


def test_su2_lattice_gauge_invariance():
    N = 5
    cfg = _cfg(N=N)
    m = oracle.su2_model(cfg)
    st = dict(_random_state(N, seed=3), a=1.0, b=0.3)
    rng = np.random.default_rng(9)
    beta = rng.uniform(0, 2 * math.pi, (N, N, N))
    gam = rng.uniform(-1.5, 1.5, (3, N, N, N))
    st2 = _gauge_transform(st, beta, gam)
    o1, o2 = oracle.su2_sync_observe(m, st), oracle.su2_sync_observe(m, st2)
    for k in ("EK", "EG", "EV", "EK_A", "EG_A", "EK_B", "EG_B"):
        assert abs(o1[k] - o2[k]) < 1e-12 * abs(o1[k]), k
    h = 0.01
    oracle.su2_vv_steps(m, st, h, "vv2", 15)
    oracle.su2_vv_steps(m, st2, h, "vv2", 15)
    st1t = _gauge_transform(st, beta, gam)
    for key in ("phi", "pi", "links", "su2", "piA", "piB"):
        assert np.max(np.abs(st1t[key] - st2[key])) < 1e-11, key
    assert abs(st["a"] - st2["a"]) < 1e-13


@pytest.mark.parametrize("integ", ["vv2", "vv4"])
def test_su2_reversibility_and_unitarity(integ):
    cfg = _cfg(N=6)
    st = oracle.su2_vacuum_ic(cfg)
    m = oracle.su2_model(cfg)
    st0 = _copy(st)
    oracle.su2_vv_steps(m, st, 0.02, integ, 25)
    assert np.max(np.abs((st["su2"] ** 2).sum(axis=1) - 1.0)) < 1e-13
    assert np.max(np.abs((st["links"] ** 2).sum(axis=1) - 1.0)) < 1e-13
    for k in ("pi", "piA", "piB"):
        st[k] = -st[k]
    st["b"] = -st["b"]
    oracle.su2_vv_steps(m, st, 0.02, integ, 25)
    for k in ("pi", "piA", "piB"):
        st[k] = -st[k]
    st["b"] = -st["b"]
    for k in ("phi", "pi", "links", "su2", "piA", "piB"):
        assert np.max(np.abs(st[k] - st0[k])) < 1e-11 * max(1.0, np.max(np.abs(st0[k]))), k
    assert abs(st["a"] - st0["a"]) < 1e-12 and abs(st["b"] - st0["b"]) < 1e-11


@pytest.mark.parametrize("integ,ratio", [("vv2", 4.0), ("vv4", 16.0)])
def test_su2_convergence_order(integ, ratio):
    cfg = _cfg(N=5, omega_over_f=1.0)
    st0 = oracle.su2_vacuum_ic(cfg)
    m = oracle.su2_model(cfg)
    res = []
    for h in (0.04, 0.02, 0.01):
        st = _copy(st0)
        oracle.su2_vv_steps(m, st, h, integ, int(round(0.4 / h)))
        res.append(st)
    for key in ("phi", "su2", "piB"):
        e1 = np.max(np.abs(res[0][key] - res[1][key]))
        e2 = np.max(np.abs(res[1][key] - res[2][key]))
        assert 0.8 * ratio < e1 / e2 < 1.25 * ratio, (integ, key, e1 / e2)


def test_su2_leapfrog_and_verlet_agree_to_second_order():
    cfg = _cfg(N=5, omega_over_f=1.0)
    st0 = oracle.su2_vacuum_ic(cfg)
    m = oracle.su2_model(cfg)
    diffs = []
    for h in (0.02, 0.01):
        n = int(round(0.4 / h))
        v = _copy(st0)
        oracle.su2_vv_steps(m, v, h, "vv2", n)
        lf = _copy(st0)
        oracle.su2_lf_startup(m, lf, h)
        oracle.su2_lf_steps(m, lf, h, n)
        diffs.append(np.max(np.abs(v["su2"] - lf["su2"])))
    assert 3.2 < diffs[0] / diffs[1] < 5.0, diffs


def test_su2_flat_space_total_energy_conserved_at_second_order():
    # a = 1: E_K + E_G + E_V + E_K^A + E_G^A + E_K^B + E_G^B is the Hamiltonian whose forces the
    # kernels are; with any relative factor wrong (current, plaquette force, Cayley angle,
    # energy normalisation) it would drift at O(1) instead of O(h^2)
    N = 5
    cfg = _cfg(N=N, expansion=False, omega_over_f=1.0, lam=0.3, e=0.7, g=0.9)
    m = oracle.su2_model(cfg)
    base = dict(_random_state(N, seed=21, amp=0.4, link_angle=1.5, emom=1.0), a=1.0, b=0.0)
    tot = lambda o: sum(o[k] for k in ("EK", "EG", "EV", "EK_A", "EG_A", "EK_B", "EG_B"))
    E0 = tot(oracle.su2_sync_observe(m, base))
    o0 = oracle.su2_sync_observe(m, base)
    assert o0["EG_B"] > 0.1 * E0 and o0["EK_B"] > 0.03 * E0 and o0["EG_A"] > 0.01 * E0
    devs = []
    for h in (0.02, 0.01):
        st = _copy(base)
        dev = 0.0
        for _ in range(int(round(0.6 / h)) // 5):
            oracle.su2_vv_steps(m, st, h, "vv2", 5)
            dev = max(dev, abs(tot(oracle.su2_sync_observe(m, st)) - E0))
        devs.append(dev / E0)
    assert devs[0] < 1e-2 and 3.2 < devs[0] / devs[1] < 5.0, devs


def test_su2_weak_nonabelian_wave_dispersion():
    # Phi = 0, one colour of B_y a plane wave along x: the links stay in one U(1) subgroup and
    # the field oscillates with the lattice frequency 2 sin(pi m/N)/dx (leapfrog map)
    N, h, nsteps, eps, mm = 10, 0.02, 60, 1e-4, 2
    cfg = _cfg(N=N, expansion=False, g=0.8, kIR=0.8, phi0=(0.0,) * 4)
    m = oracle.su2_model(cfg)
    dx = m.dx
    x = np.arange(N)[:, None, None] * np.ones((1, N, N))
    mode = np.cos(2 * math.pi * mm * x / N + 0.3)
    B = eps * mode
    su2 = np.zeros((3, 4, N, N, N))
    su2[:, 0] = 1.0
    # U_y = exp(-i g dx B T_1) = cos(g dx B / 2) - i sin(g dx B / 2) sigma_1
    su2[1, 0] = np.cos(m.g * dx * B / 2)
    su2[1, 1] = -np.sin(m.g * dx * B / 2)
    links = np.zeros((3, 2, N, N, N))
    links[:, 0] = 1.0
    st = {"phi": np.zeros((4, N, N, N)), "pi": np.zeros((4, N, N, N)), "links": links, "su2": su2,
          "piA": np.zeros((3, N, N, N)), "piB": np.zeros((3, 3, N, N, N)), "a": 1.0, "b": 0.0}
    oracle.su2_lf_steps(m, st, h, nsteps)
    w2 = (2.0 * math.sin(math.pi * mm / N) / dx) ** 2
    Lm = np.array([[1 - h * h * w2, h], [-h * w2, 1.0]])
    Bf, Pf = np.linalg.matrix_power(Lm, nsteps) @ np.array([1.0, 0.0])
    By = -2.0 * np.arcsin(st["su2"][1, 1]) / (m.g * dx)
    assert np.max(np.abs(By - eps * Bf * mode)) < 1e-6 * eps
    assert np.max(np.abs(st["piB"][1, 0] - eps * Pf * mode)) < 1e-6 * eps * math.sqrt(w2)
    others = np.delete(st["piB"].reshape(9, -1), 3, axis=0)
    assert np.max(np.abs(others)) < 1e-12 * eps


def test_su2_homogeneous_limit_against_ode():
    # links 1, no electric fields, homogeneous Phi with four equal components c: the radial
    # mode psi = 2 sqrt(2) c obeys psi'' + 3 H psi' + lam psi^3 = 0, rho = psi'^2/2 + lam psi^4/4
    from scipy.integrate import solve_ivp

    lam, fmp, psi0, T, alpha = 1.0, 2.0, 0.8, 1.0, 0.0
    cfg = dict(_cfg(N=4, alpha=alpha), fstar_over_mp=fmp, lam=lam)
    m = oracle.su2_model(cfg)

    def rhs(t, y):
        p, v, aa, eta = y
        H = fmp * math.sqrt((v * v / 2 + lam * p ** 4 / 4) / 3.0)
        return [v, -3 * H * v - lam * p ** 3, aa * H, aa ** (-alpha)]

    ev = lambda t, y: y[3] - T
    ev.terminal = True
    sol = solve_ivp(rhs, [0, 50], [psi0, 0.0, 1.0, 0.0], method="DOP853", rtol=1e-13, atol=1e-14, events=ev)
    p_ode, _, a_ode, _ = sol.y_events[0][0]
    errs = []
    for h in (0.01, 0.005):
        links = np.zeros((3, 2, 4, 4, 4))
        links[:, 0] = 1.0
        su2 = np.zeros((3, 4, 4, 4, 4))
        su2[:, 0] = 1.0
        c = psi0 / (2 * math.sqrt(2.0))
        st = {"phi": np.full((4, 4, 4, 4), c), "pi": np.zeros((4, 4, 4, 4)), "links": links, "su2": su2,
              "piA": np.zeros((3, 4, 4, 4)), "piB": np.zeros((3, 3, 4, 4, 4)), "a": 1.0,
              "b": fmp * math.sqrt(lam * psi0 ** 4 / 4 / 3.0)}
        oracle.su2_lf_startup(m, st, h)
        oracle.su2_lf_steps(m, st, h, int(round(T / h)))
        errs.append((abs(st["a"] - a_ode), abs(st["phi"][0, 0, 0, 0] * 2 * math.sqrt(2.0) - p_ode)))
    for j in range(2):
        assert 3.0 < errs[0][j] / errs[1][j] < 5.0, errs
    assert max(errs[1]) < 1e-4


def _u1_from_upper(st, e):
    """The U(1) model's state made of the doublet's upper component and U(1) sector."""
    return {"phi": st["phi"][:2].copy(), "pi": st["pi"][:2].copy(), "links": st["links"].copy(),
            "piA": st["piA"].copy(), "a": st["a"], "b": st["b"]}


@pytest.mark.parametrize("integ", ["lf2", "vv2"])
def test_su2_reduces_to_u1_for_the_upper_component(integ):
    # Phi_1 = 0, SU(2) links 1, pi_B = 0: with the SU(2) coupling g -> 0 its field is sourced at
    # O(g) and acts back at O(g^2), so the U(1) sector and Phi_0 follow the U(1) model
    N = 6
    cfg = _cfg(N=N, g=1e-6, omega_over_f=1.0)
    m = oracle.su2_model(cfg)
    rs = _random_state(N, seed=5, amp=0.3, link_angle=1.0, emom=0.4)
    rs["phi"][2:] = 0.0
    rs["pi"][2:] = 0.0
    rs["su2"][:] = 0.0
    rs["su2"][:, 0] = 1.0
    rs["piB"][:] = 0.0
    st = dict(rs, a=1.0, b=0.7)
    ucfg = dict(cfg, model="u1")
    mu = oracle.u1_model(ucfg)
    su = _u1_from_upper(st, cfg["e"])
    h = 0.01
    if integ == "lf2":
        oracle.su2_lf_startup(m, st, h)
        oracle.u1_lf_startup(mu, su, h)
        oracle.su2_lf_steps(m, st, h, 30)
        oracle.u1_lf_steps(mu, su, h, 30)
        o, ou = oracle.su2_lf_observe(m, st, h), oracle.u1_lf_observe(mu, su, h)
    else:
        oracle.su2_vv_steps(m, st, h, "vv2", 30)
        oracle.u1_vv_steps(mu, su, h, "vv2", 30)
        o, ou = oracle.su2_sync_observe(m, st), oracle.u1_sync_observe(mu, su)
    for k in ("phi", "pi"):
        assert np.max(np.abs(st[k][:2] - su[k])) < 1e-10, k
        assert np.max(np.abs(st[k][2:])) == 0.0
    for k in ("links", "piA"):
        assert np.max(np.abs(st[k] - su[k])) < 1e-10, k
    for k in ("a", "b", "EK", "EG", "EV", "EK_A", "EG_A"):
        assert abs(o[k] - ou[k]) < 1e-10 * abs(ou[k]), k
    assert o["EK_B"] < 1e-9 * o["EK"]


@pytest.mark.parametrize("integ", ["lf2", "vv2"])
def test_su2_sigma3_subgroup_acts_as_u1_of_charge_g_over_2(integ):
    # Phi_1 = 0, SU(2) links exp(i th sigma_3), pi_B along T_3 only, U(1) coupling e -> 0 and
    # V = 1, pi_A = 0: the upper component sees exp(i th); current, plaquette force, Cayley
    # drift and energies then equal the U(1) model's with e' = g/2 (th = U(1) phase)
    N = 6
    g = 0.8
    cfg = _cfg(N=N, e=1e-7, g=g, omega_over_f=1.0)
    m = oracle.su2_model(cfg)
    rs = _random_state(N, seed=8, amp=0.3)
    rs["phi"][2:] = 0.0
    rs["pi"][2:] = 0.0
    rs["links"][:] = 0.0
    rs["links"][:, 0] = 1.0
    rs["piA"][:] = 0.0
    rng = np.random.default_rng(2)
    th = rng.uniform(-0.5, 0.5, (3, N, N, N))
    rs["su2"][:] = 0.0
    rs["su2"][:, 0] = np.cos(th)
    rs["su2"][:, 3] = np.sin(th)
    rs["piB"][:] = 0.0
    rs["piB"][:, 2] = rng.uniform(-0.4, 0.4, (3, N, N, N))
    st = dict(rs, a=1.0, b=0.7)
    ucfg = dict(cfg, model="u1", e=g / 2)
    mu = oracle.u1_model(ucfg)
    su = {"phi": st["phi"][:2].copy(), "pi": st["pi"][:2].copy(),
          "links": np.stack([np.cos(th), np.sin(th)], axis=1), "piA": st["piB"][:, 2].copy(), "a": 1.0, "b": 0.7}
    h = 0.01
    if integ == "lf2":
        oracle.su2_lf_startup(m, st, h)
        oracle.u1_lf_startup(mu, su, h)
        oracle.su2_lf_steps(m, st, h, 30)
        oracle.u1_lf_steps(mu, su, h, 30)
        o, ou = oracle.su2_lf_observe(m, st, h), oracle.u1_lf_observe(mu, su, h)
    else:
        oracle.su2_vv_steps(m, st, h, "vv2", 30)
        oracle.u1_vv_steps(mu, su, h, "vv2", 30)
        o, ou = oracle.su2_sync_observe(m, st), oracle.u1_sync_observe(mu, su)
    assert np.max(np.abs(st["phi"][:2] - su["phi"])) < 1e-9
    assert np.max(np.abs(st["su2"][:, 0] - su["links"][:, 0])) < 1e-9
    assert np.max(np.abs(st["su2"][:, 3] - su["links"][:, 1])) < 1e-9
    assert np.max(np.abs(st["su2"][:, 1:3])) < 1e-12
    assert np.max(np.abs(st["piB"][:, 2] - su["piA"])) < 1e-9
    for ka, kb in (("EK_B", "EK_A"), ("EG_B", "EG_A"), ("EK", "EK"), ("EG", "EG"), ("b", "b")):
        assert abs(o[ka] - ou[kb]) < 1e-9 * abs(ou[kb]), ka


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_su2_hubble_constraint_with_gauge_energy_converges(alpha):
    # gauge-dominated state: the (alpha - 1)(E_K^A + E_G^A + E_K^B + E_G^B) term of K_a is
    # needed for the constraint residual to fall as h^2
    N = 5
    cfg = _cfg(N=N, alpha=alpha, omega_over_f=1.0, lam=0.05)
    m = oracle.su2_model(cfg)
    base = dict(_random_state(N, seed=11, amp=0.05, link_angle=1.5, emom=1.0), a=1.0, b=1.0)
    o = oracle.su2_sync_observe(m, base)
    assert o["EK_B"] + o["EG_B"] > 3 * (o["EK"] + o["EG"] + o["EV"])
    base["b"] = math.sqrt(m.fmp2 / 3.0 * o["rho"])
    hcs = []
    for h in (0.01, 0.005):
        st = _copy(base)
        oracle.su2_vv_steps(m, st, h, "vv2", int(round(0.5 / h)))
        hcs.append(oracle.su2_sync_observe(m, st)["hc"])
    assert hcs[0] < 1e-2 and 3.0 < hcs[0] / hcs[1] < 5.0, hcs


def test_su2_hubble_constraint_has_no_lattice_spacing_floor():
    # the kernels are the forces of the energies (left-invariant electric fields generate the
    # link motion), so the Friedmann-constraint violation falls as h^4 with VV4 to the 1e-9
    # level, with no floor of order dx at fixed lattice spacing
    N = 5
    cfg = _cfg(N=N, alpha=0.5, omega_over_f=1.0, lam=0.05)
    m = oracle.su2_model(cfg)
    base = dict(_random_state(N, seed=11, amp=0.05, link_angle=1.5, emom=1.0), a=1.0, b=1.0)
    base["b"] = math.sqrt(m.fmp2 / 3.0 * oracle.su2_sync_observe(m, base)["rho"])
    hcs = []
    for h in (0.01, 0.005, 0.0025):
        st = _copy(base)
        oracle.su2_vv_steps(m, st, h, "vv4", int(round(0.5 / h)))
        hcs.append(oracle.su2_sync_observe(m, st)["hc"])
    assert hcs[-1] < 1e-8
    for k in range(2):
        assert 13.0 < hcs[k] / hcs[k + 1] < 19.0, hcs
