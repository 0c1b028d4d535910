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


# --------------------------------------------------------------------------
# Initial state of the charged scalar (Sec. 7.1, 7.2), pinned from its output
# --------------------------------------------------------------------------
def _u1_potential_curvature(lam, m2, pb, n, eps=1e-4):
    """d^2 V / d phi_n^2 of V = lam |phi|^4 + m2 |phi|^2, |phi|^2 = (phi_0^2 + phi_1^2)/2,
    by a central difference of the potential itself (not of a closed form)."""
    def V(p0, p1):
        r2 = 0.5 * (p0 * p0 + p1 * p1)
        return lam * r2 * r2 + m2 * r2

    p = list(pb)
    vals = []
    for d in (-eps, 0.0, eps):
        q = list(p)
        q[n] += d
        vals.append(V(*q))
    return (vals[0] - 2 * vals[1] + vals[2]) / (eps * eps)


def _modes_of(field, N):
    """f(n~) = sum_n exp(+2 pi i n~.n/N) f(n) through numpy's inverse FFT."""
    return np.fft.ifftn(field) * N ** 3


def _half_space(N):
    """One member of every +-n~ pair that is not its own partner, by a rule of
    this test (smaller linear index of the two)."""
    idx = np.arange(N)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    lin = (I * N + J) * N + K
    par = ((-I) % N * N + (-J) % N) * N + (-K) % N
    return lin < par


def _u1_ic_decompose(cfg, st):
    """Left/right movers L_n, R_n of each real component (Sec. 7.2 form
    df = (L + R)/sqrt 2, df' = c i w (L - R)/sqrt 2 - H df) recovered from the
    output state, with every ingredient computed here: w_k^2 = k^2 + a^2 d2V,
    H from the homogeneous Friedmann equation, c = a^{-(1-alpha)}."""
    N = cfg["N"]
    kIR, al, a = cfg["kIR"], cfg["alpha"], cfg["a0"]
    dx = 2 * math.pi / (kIR * N)
    lam, m2 = cfg["lam"], cfg["m2"][0]
    pb, db = cfg["phi0"], cfg["dphi0"]
    r2 = 0.5 * (pb[0] ** 2 + pb[1] ** 2)
    rho_h = (db[0] ** 2 + db[1] ** 2) / (2 * a ** (2 * al)) + lam * r2 * r2 + m2 * r2
    H = math.sqrt(cfg["fstar_over_mp"] ** 2 / 3 * a ** (2 * al + 2) * rho_h) / a
    f = np.fft.fftfreq(N) * N
    F1, F2, F3 = np.meshgrid(f, f, f, indexing="ij")
    k = kIR * np.sqrt(F1 ** 2 + F2 ** 2 + F3 ** 2)
    P0 = cfg["omega_over_f"] ** 2 * (N / dx) ** 3
    out = []
    for n in range(2):
        comp = math.sqrt(2.0) * st["phi"][n] - pb[n]          # phi = (phi_0 + i phi_1)/sqrt 2
        dcomp = math.sqrt(2.0) * st["pi"][n] / a ** (3 - al) - db[n]   # pi = a^{3-alpha} phi'
        Fm, Fd = _modes_of(comp, N), _modes_of(dcomp, N)
        w = np.sqrt(k * k + a * a * _u1_potential_curvature(lam, m2, pb, n))
        P = P0 / (2 * a * a * w)
        G = (Fd + H * Fm) / (a ** (-(1 - al)) * 1j * np.where(w > 0, w, 1.0))
        out.append(dict(F=Fm, Fd=Fd, L=(Fm + G) / math.sqrt(2), R=(Fm - G) / math.sqrt(2), P=P, w=w, H=H))
    return out


def _u1_ic_cfg(seed, N=12):
    return dict(model="u1", nf=2, N=N, kIR=0.3, dt=0.01, alpha=1.0, fstar_over_mp=2.0, omega_over_f=0.05,
                m2=(0.0, 0.0), lam=1.0, q=0.0, e=0.5, phi0=(0.9, 0.4), dphi0=(0.0, 0.0), expansion=True,
                seed=seed, a0=1.0)


@pytest.mark.parametrize("a0", [1.0, 2.0])
def test_u1_vacuum_ic_movers_obey_the_charge_constraints_mode_by_mode(a0):
    # |l_n| = |r_n| and th_1^r = th_0^r + th_1^l - th_0^l at every mode (Sec. 7.2): only
    # true if the test's w_k (with m2_eff,n = d2V/dphi_n^2), H, the 1/sqrt 2 of the complex
    # field and pi = a^{3-alpha} phi' all match what the generator used.  alpha = 1, so that
    # a0 = 2 tests the powers of a without the a^{+-(1-alpha)} of the derivative modes,
    # which the paper writes both ways (Sec. 7.1 against Sec. 7.2) and which is 1 here.
    cfg = dict(_u1_ic_cfg(5), a0=a0)
    d = _u1_ic_decompose(cfg, oracle.u1_vacuum_ic(cfg))
    hs = _half_space(cfg["N"])
    scale = np.sqrt(d[0]["P"][hs]).max()
    for n in range(2):
        L, R = d[n]["L"][hs], d[n]["R"][hs]
        assert np.max(np.abs(np.abs(L) - np.abs(R))) < 1e-9 * scale, n
        assert np.abs(L).min() > 0
    ph = d[1]["R"][hs] * d[0]["L"][hs] / (d[0]["R"][hs] * d[1]["L"][hs])   # e^{i(th1r - th0r - th1l + th0l)}
    assert np.max(np.abs(ph - 1.0)) < 1e-8


def test_u1_vacuum_ic_mode_statistics():
    # Ensemble over 48 seeds of |df_n|^2 / P_n (Rayleigh moduli: mean 1), of the derivative
    # modes |df'_n|^2 / ((c^2 w^2 + H^2) P_n), and of the fourth moment of Re df_n.
    # With |l| = |r| a mode is |l| (e^{i th_l} + e^{i th_r})/sqrt 2, whose real part has
    # kurtosis 9/2 (E|l|^4 = 2 P^2, E(Re Z)^2 = 1, E(Re Z)^4 = 9/4 for Z = e^{ia} + e^{ib}),
    # not the 3 of independent Gaussian movers.
    N = 12
    hs = _half_space(N)
    r = [[], []]
    rd = [[], []]
    z = [[], []]
    for s in range(48):
        cfg = _u1_ic_cfg(1000 + s, N)
        d = _u1_ic_decompose(cfg, oracle.u1_vacuum_ic(cfg))
        for n in range(2):
            P, w, H = d[n]["P"][hs], d[n]["w"][hs], d[n]["H"]
            r[n].append(np.abs(d[n]["F"][hs]) ** 2 / P)
            rd[n].append(np.abs(d[n]["Fd"][hs]) ** 2 / ((w * w + H * H) * P))
            z[n].append(d[n]["F"][hs].real / np.sqrt(P / 2))
    for n in range(2):
        for arr in (np.concatenate(r[n]), np.concatenate(rd[n])):
            assert abs(arr.mean() - 1) < 3 * arr.std() / math.sqrt(arr.size), (n, arr.mean())
        zz = np.concatenate(z[n])
        assert abs(np.mean(zz ** 2) - 1) < 0.03
        kurt = np.mean(zz ** 4) / np.mean(zz ** 2) ** 2
        assert abs(kurt - 4.5) < 0.3, (n, kurt)


def test_u1_vacuum_ic_statistics_see_a_wrong_effective_mass():
    # the statistics above are sensitive to m2_eff: the low shells of component 0 at
    # m2_eff = lam (s + 2 phi_0^2) against lam s (the curvature of |phi|^4 along |phi| only)
    N = 12
    hs = _half_space(N)
    f = np.fft.fftfreq(N) * N
    F1, F2, F3 = np.meshgrid(f, f, f, indexing="ij")
    low = (np.sqrt(F1 ** 2 + F2 ** 2 + F3 ** 2) <= 2.0)[hs]
    good, bad = [], []
    for s in range(48):
        cfg = _u1_ic_cfg(2000 + s, N)
        d = _u1_ic_decompose(cfg, oracle.u1_vacuum_ic(cfg))[0]
        P = d["P"][hs][low]
        k2 = (d["w"][hs][low]) ** 2 - _u1_potential_curvature(1.0, 0.0, cfg["phi0"], 0)
        Pbad = P * d["w"][hs][low] / np.sqrt(k2 + 1.0 * (0.9 ** 2 + 0.4 ** 2))
        good.append(np.abs(d["F"][hs][low]) ** 2 / P)
        bad.append(np.abs(d["F"][hs][low]) ** 2 / Pbad)
    g, b = np.concatenate(good), np.concatenate(bad)
    assert abs(g.mean() - 1) < 3 * g.std() / math.sqrt(g.size)
    assert abs(b.mean() - 1) > 6 * b.std() / math.sqrt(b.size)


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_u1_initial_gauss_law_at_a0_not_one(alpha):
    # the kicks conserve sum_i D-_i piA_i - 2e (f/w)^2 Im[conj phi pi] with no power of a,
    # so the initial link momenta must solve exactly that at any a0 (Sec. 7.2 with a0 != 1)
    cfg = dict(_cfg(N=8, alpha=alpha), a0=2.0)
    st = oracle.u1_vacuum_ic(cfg)
    m = oracle.u1_model(cfg)
    assert oracle.u1_sync_observe(m, st)["gauss"] < 1e-12
    h = 0.01
    vv = _copy(st)
    oracle.u1_vv_steps(m, vv, h, "vv2", 20)
    assert oracle.u1_sync_observe(m, vv)["gauss"] < 1e-12
    oracle.u1_lf_startup(m, st, h)
    oracle.u1_lf_steps(m, st, h, 20)
    assert oracle.u1_lf_observe(m, st, h)["gauss"] < 1e-12


# --------------------------------------------------------------------------
# U(1) spectra (Sec. 5.4.2)
# --------------------------------------------------------------------------
def test_u1_spectra_parseval():
    # sum_b S_b = N^3 sum_n sum_c f_c(n)^2 for the complex scalar, its momentum, E and B
    cfg = _cfg(N=10)
    rs = synth.random_u1_state(10, seed=4, amp=0.3, link_angle=1.2, emom=0.4)
    st = dict(rs, a=1.7, b=0.2)
    N = 10
    for which, parts in (("phi", st["phi"]), ("pi", st["pi"]), ("E", st["piA"] * 1.7 ** (-(1 - cfg["alpha"])))):
        sp = oracle.u1_spectrum(cfg, st, which)
        assert abs(sp["S"].sum() - N ** 3 * np.sum(parts ** 2)) < 1e-10 * sp["S"].sum(), which
    # B from the plaquettes, built here with complex numbers from the phases
    th = np.arctan2(st["links"][:, 1], st["links"][:, 0])
    dx = 2 * math.pi / (cfg["kIR"] * N)
    Bsq = 0.0
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        phi_jk = th[j] + np.roll(th[k], -1, axis=j) - np.roll(th[j], -1, axis=k) - th[k]
        Bsq += np.sum((np.sin(phi_jk) / (cfg["e"] * dx * dx)) ** 2)
    sp = oracle.u1_spectrum(cfg, st, "B")
    assert abs(sp["S"].sum() - N ** 3 * Bsq) < 1e-10 * sp["S"].sum()


@pytest.mark.parametrize("model", ["u1", "u1nc"])
def test_u1_magnetic_spectrum_single_mode(model):
    # A_y = eps cos(2 pi m x/N + psi): B_z = D+_x A_y is one lattice wave, all its power in
    # shell m with S_m = N^6 eps^2 k_lat^2 / 2, k_lat = 2 sin(pi m/N)/dx (compact: up to
    # the O((e dx^2 eps k)^2) of sin(Phi) against Phi)
    N, m, eps = 12, 3, 1e-4
    cfg = dict(_cfg(N=N), model=model)
    dx = 2 * math.pi / (cfg["kIR"] * N)
    x = np.arange(N)[:, None, None] * np.ones((1, N, N))
    A = np.zeros((3, N, N, N))
    A[1] = eps * np.cos(2 * math.pi * m * x / N + 0.4)
    if model == "u1":
        links = np.zeros((3, 2, N, N, N))
        th = -cfg["e"] * dx * A
        links[:, 0], links[:, 1] = np.cos(th), np.sin(th)
    else:
        links = A
    st = {"phi": np.zeros((2, N, N, N)), "pi": np.zeros((2, N, N, N)), "links": links,
          "piA": np.zeros((3, N, N, N)), "a": 1.0, "b": 0.0}
    sp = oracle.u1_spectrum(cfg, st, "B")
    klat = 2 * math.sin(math.pi * m / N) / dx
    expect = N ** 6 * eps ** 2 * klat ** 2 / 2
    tol = 1e-10 if model == "u1nc" else 1e-6
    assert abs(sp["S"][m] - expect) < tol * expect
    others = np.delete(sp["S"], m)
    assert np.max(others) < tol * expect


def test_u1_electric_spectrum_single_mode_and_scale_factor():
    # pi_A,x = eps cos(2 pi m y/N): shell m holds N^6 eps^2/2, times a^{-2(1-alpha)}
    N, m, eps = 12, 4, 0.3
    cfg = _cfg(N=N, alpha=0.5)
    y = np.arange(N)[None, :, None] * np.ones((N, 1, N))
    piA = np.zeros((3, N, N, N))
    piA[0] = eps * np.cos(2 * math.pi * m * y / N)
    st = {"phi": np.zeros((2, N, N, N)), "pi": np.zeros((2, N, N, N)),
          "links": np.zeros((3, 2, N, N, N)), "piA": piA, "a": 2.0, "b": 0.0}
    sp = oracle.u1_spectrum(cfg, st, "E")
    expect = N ** 6 * eps ** 2 / 2 / 2.0
    assert abs(sp["S"][m] - expect) < 1e-12 * expect
    assert np.max(np.delete(sp["S"], m)) < 1e-12 * expect
