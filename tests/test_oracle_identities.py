"""Pins of the oracle's single-node arithmetic against identities the paper states.

Each check compares the oracle with a fact fixed by the paper or by the mathematics, not
with a retyping of the oracle's own formula:
  * the velocity moments of the equilibria, forcing and source terms that the
    Chapman-Enskog analysis relies on (Sec. 3.2 moment list, App. A moment lists);
  * the closed forms of s_0 and F_0 (App. A, last equation);
  * the lattice of Sec. 3.1 (isotropy of the weights up to fourth order);
  * the defining implicit equation of the quadratic drag solve (Sec. 3.1);
  * recovery of S and grad T from states built with a prescribed non-equilibrium part
    (Eqs. ShearEqCom, SonaT), including the direct formula for u . grad T = 0 and the
    determinant of Eq. detMatr along the eigen-directions of <M>.
"""
import numpy as np
import pytest

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def lat(oracle_mod):
    cx, cy, w = oracle_mod.lattice()
    return np.stack([cx, cy], 1).astype(np.float64), w


def _cfg(rng, **kw):
    cfg = {"nx": 8, "ny": 8, "periodic_x": 1, "periodic_y": 1,
           "tau_f": rng.uniform(0.6, 1.5), "tau_T": rng.uniform(0.6, 1.5),
           "A": rng.uniform(-0.2, 0.05), "B": rng.uniform(-0.2, 0.05),
           "sigma": rng.uniform(0.8, 1.3), "Q": rng.uniform(-1e-3, 1e-3),
           "Da": 10 ** rng.uniform(-3, -1), "Ra": 1e4, "Pr": 1.0, "J": 1.0,
           "eps": rng.uniform(0.3, 1.0)}
    cfg.update(kw)
    return cfg


def test_lattice_matches_paper(lat):
    c, w = lat
    expect = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    assert np.array_equal(c, expect)
    assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-16)
    # isotropy up to fourth order with cs^2 = 1/3
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * np.eye(2), atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    d = np.eye(2)
    iso4 = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-16)


@pytest.mark.parametrize("seed", range(20))
def test_moment_identities(oracle_mod, lat, seed):
    c, w = lat
    rng = np.random.default_rng(seed)
    cfg = _cfg(rng)
    d = oracle_mod.derived(cfg)
    eps, T = cfg["eps"], rng.uniform(0.0, 2.0)
    u = rng.uniform(-0.1, 0.1, 2)
    p = rng.uniform(-0.01, 0.01)
    S = rng.uniform(-0.01, 0.01, (2, 2))
    S = S + S.T                      # symmetric, with a trace
    gT = rng.uniform(-0.05, 0.05, 2)
    F = rng.uniform(-1e-3, 1e-3, 2)
    t = oracle_mod.node_terms(cfg, eps, T, u[0], u[1], p, S[0, 0], S[0, 1], S[1, 1],
                              gT[0], gT[1], F[0], F[1])
    rho0, sig, tf, tT, Q = 1.0, cfg["sigma"], cfg["tau_f"], cfg["tau_T"], cfg["Q"]
    A, B = d["A"], d["B"]
    I = np.eye(2)
    m0 = lambda x: x.sum()
    m1 = lambda x: np.einsum("i,ia->a", x, c)
    m2 = lambda x: np.einsum("i,ia,ib->ab", x, c, c)
    m3 = lambda x: np.einsum("i,ia,ib,ic->abc", x, c, c, c)
    delta_u = (np.einsum("a,bc->abc", u, I) + np.einsum("b,ac->abc", u, I)
               + np.einsum("c,ab->abc", u, I))
    tol = 1e-15
    # flow EDF (App. A, moments of f^{e(0)} and f^{e(1)})
    fe0, r = t["feq0"], t["r"]
    assert abs(m0(fe0) - rho0) < tol
    assert np.allclose(m1(fe0), rho0 * u, atol=tol)
    assert np.allclose(m2(fe0), eps * p * I + rho0 * np.outer(u, u) / eps, atol=tol)
    assert np.allclose(m3(fe0), CS2 * rho0 * delta_u, atol=tol)
    assert abs(m0(r)) < tol and np.allclose(m1(r), 0, atol=tol)
    assert np.allclose(m2(rho0 * r), CS2 * rho0 * A * S, atol=tol)
    # closed forms of s_0 (via f_0^{e(0)}) and F_0
    s0 = -w[0] / (2 * eps * CS2) * (u @ u)
    assert abs(fe0[0] - (rho0 - (1 - w[0]) * eps * p / CS2 + rho0 * s0)) < tol
    F0 = -w[0] * (1 - 1 / (2 * tf)) * (u @ F) / (eps * CS2)
    assert abs(t["F"][0] - F0) < tol
    # forcing term (App. A, moments of F_i)
    Fi = t["F"]
    assert abs(m0(Fi)) < tol
    assert np.allclose(m1(Fi), (1 - 1 / (2 * tf)) * rho0 * F, atol=tol)
    assert np.allclose(m2(Fi), (1 - 1 / (2 * tf)) * rho0 * (np.outer(u, F) + np.outer(F, u)) / eps,
                       atol=tol)
    # temperature EDF (Sec. 3.2 moment list)
    ge0, gB = t["geq0"], t["gB"]
    assert abs(m0(ge0) - sig * T) < tol
    assert np.allclose(m1(ge0), T * u, atol=tol)
    assert np.allclose(m2(ge0), T * np.outer(u, u) / eps + CS2 * sig * T * I + eps * p * T / rho0 * I,
                       atol=tol)
    assert np.allclose(m3(ge0), CS2 * T * delta_u, atol=tol)
    assert abs(m0(gB)) < tol
    assert np.allclose(m1(gB), sig * CS2 * B * gT, atol=tol)
    assert np.allclose(m2(gB), 0, atol=tol)
    # thermal sources
    P, Qi = t["P"], t["Q"]
    assert abs(m0(P)) < tol
    assert np.allclose(m1(P), (1 - 1 / (2 * tT)) * (T * F + eps * p * gT / rho0
                                                   + (1 / eps - 1 / sig) * u * (u @ gT)), atol=tol)
    assert np.allclose(m2(P), 0, atol=tol)
    assert abs(m0(Qi) - (1 - 1 / (2 * tT)) * Q) < tol
    assert np.allclose(m1(Qi), (1 - 1 / (2 * tT)) * u * Q / sig, atol=tol)


def _drag_F(cfg, d, eps, u, G):
    """Total force of Eq. ForceEq (Ergun F_eps) for the drag-inversion pin."""
    Feps = 1.75 / np.sqrt(150 * eps ** 3)
    return -eps * d["nu"] / d["K"] * u - eps * Feps / np.sqrt(d["K"]) * np.linalg.norm(u) * u + eps * G


@pytest.mark.parametrize("seed", range(10))
def test_drag_solve_satisfies_implicit_definition(oracle_mod, lat, seed):
    """u = sum c f / rho0 + F(u)/2 with F nonlinear in u (Sec. 3.1): build f with the
    first moment that a chosen u requires and recover u."""
    c, w = lat
    rng = np.random.default_rng(100 + seed)
    cfg = _cfg(rng, Q=0.0, Ra=0.0, A=0.0, B=0.0, ax=rng.uniform(-1e-4, 1e-4), ay=rng.uniform(-1e-4, 1e-4))
    d = oracle_mod.derived(cfg)
    eps = cfg["eps"]
    u = rng.uniform(-0.08, 0.08, 2)
    G = np.array([cfg["ax"], cfg["ay"]])
    j = u - 0.5 * _drag_F(cfg, d, eps, u, G)          # required sum_i c_i f_i (rho0 = 1)
    f = np.zeros(9)
    f[0] = 1.0
    f[1], f[3] = 0.5 * j[0] + 0.01, -0.5 * j[0] + 0.01
    f[2], f[4] = 0.5 * j[1] + 0.01, -0.5 * j[1] + 0.01
    g = w * 0.5
    m = oracle_mod.node_macro(cfg, eps, f, g)
    assert abs(m["ux"] - u[0]) < 1e-15 and abs(m["uy"] - u[1]) < 1e-15
    Fm = _drag_F(cfg, d, eps, u, G)
    assert abs(m["Fx"] - Fm[0]) < 1e-16 and abs(m["Fy"] - Fm[1]) < 1e-16


def _base_state(oracle_mod, cfg, eps, p, u, T):
    t = oracle_mod.node_terms(cfg, eps, T, u[0], u[1], p, 0, 0, 0, 0, 0, 0, 0)
    return t["feq0"], t["geq0"]


@pytest.mark.parametrize("seed", range(10))
def test_shear_rate_from_nonequilibrium_part(oracle_mod, lat, seed):
    """With no force, S = sum c c (f - f^{e(0)}) / (cs^2 rho0 (A - tau_f)) (Eq. ShearEqCom):
    a state f^{e(0)} + Delta with a prescribed traceless second moment of Delta returns S,
    and leaves p, u and T unchanged."""
    c, w = lat
    rng = np.random.default_rng(200 + seed)
    cfg = _cfg(rng, Da=float("inf"), Q=0.0, Ra=0.0, F_eps=0.0)
    d = oracle_mod.derived(cfg)
    eps, p, T = cfg["eps"], rng.uniform(-0.01, 0.01), rng.uniform(0, 1)
    u = rng.uniform(-0.05, 0.05, 2)
    St = rng.uniform(-0.01, 0.01, (2, 2))
    St = St + St.T
    St -= 0.5 * np.trace(St) * np.eye(2)
    X = CS2 * (d["A"] - cfg["tau_f"]) * St
    delta = w * (np.einsum("ab,ia,ib->i", X, c, c) - CS2 * np.trace(X)) / (2 * CS2 ** 2)
    f0, g0 = _base_state(oracle_mod, cfg, eps, p, u, T)
    m = oracle_mod.node_macro(cfg, eps, f0 + delta, g0)
    assert abs(m["Sxx"] - St[0, 0]) < 1e-14
    assert abs(m["Sxy"] - St[0, 1]) < 1e-14
    assert abs(m["Syy"] - St[1, 1]) < 1e-14
    assert abs(m["p"] - p) < 1e-15 and abs(m["ux"] - u[0]) < 1e-15 and abs(m["T"] - T) < 1e-15


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("orient", ["perp", "par"])
def test_temperature_gradient_eigendirections(oracle_mod, lat, seed, orient):
    """grad T from <M> grad T = <N> (Eqs. SonaT, MatrM, MatrN): for N perpendicular to u the
    direct formula with divisor cs^2 sigma (B - tau_T) - eps p / (2 rho0) holds; for N
    parallel to u the divisor loses (1/eps - 1/sigma)|u|^2 / 2, the second factor of
    Eq. detMatr."""
    c, w = lat
    rng = np.random.default_rng(300 + seed)
    cfg = _cfg(rng, Da=float("inf"), Q=0.0, Ra=0.0, F_eps=0.0, sigma=1.0)
    d = oracle_mod.derived(cfg)
    eps, p, T = cfg["eps"], rng.uniform(-0.01, 0.01), rng.uniform(0, 1)
    u = rng.uniform(-0.1, 0.1, 2)
    uhat = u / np.linalg.norm(u)
    dirv = np.array([-uhat[1], uhat[0]]) if orient == "perp" else uhat
    N = rng.uniform(0.5, 2.0) * 1e-3 * dirv
    dg = w * (c @ N) / CS2                  # sum dg = 0, sum c dg = N
    f0, g0 = _base_state(oracle_mod, cfg, eps, p, u, T)
    m = oracle_mod.node_macro(cfg, eps, f0, g0 + dg)
    a = CS2 * cfg["sigma"] * (d["B"] - cfg["tau_T"]) - eps * p / 2
    if orient == "par":
        a -= 0.5 * (1 / eps - 1 / cfg["sigma"]) * (u @ u)
    assert np.allclose([m["dTdx"], m["dTdy"]], N / a, rtol=1e-13, atol=1e-17)
    assert abs(m["T"] - T) < 1e-15


@pytest.mark.parametrize("seed", range(10))
def test_collision_conserves_mass_and_balances_energy(oracle_mod, lat, seed):
    """sum f* = rho0, sum c f* = rho0 (u + F/2), sum g* = sigma T + Q/2 follow from the
    moment lists and sigma T = sum g + Q/2 (Sec. 3.2)."""
    c, w = lat
    rng = np.random.default_rng(400 + seed)
    cfg = _cfg(rng, ax=rng.uniform(-1e-4, 1e-4), ay=rng.uniform(-1e-4, 1e-4))
    eps = cfg["eps"]
    f = w * (1 + rng.uniform(-0.05, 0.05, 9))
    f[0] = 1.0 - f[1:].sum() + rng.uniform(-1e-3, 1e-3)
    g = w * (0.5 + rng.uniform(-0.05, 0.05, 9))
    m = oracle_mod.node_macro(cfg, eps, f, g)
    fo, go = oracle_mod.node_collide(cfg, eps, f, g)
    tf = cfg["tau_f"]
    assert abs(fo.sum() - (f.sum() - (f.sum() - 1.0) / tf)) < 1e-15
    mom = c.T @ fo
    assert np.allclose(mom, np.array([m["ux"], m["uy"]]) + 0.5 * np.array([m["Fx"], m["Fy"]]),
                       atol=1e-15)
    assert abs(go.sum() - (cfg["sigma"] * m["T"] + 0.5 * cfg["Q"])) < 1e-15


def test_uniformly_accelerating_flow_has_no_shear(oracle_mod):
    """A porous flow that is uniform in space and accelerates under an oblique body force
    (Darcy and Forchheimer drag on) has no velocity gradient.  Its non-equilibrium second
    moment is -(u F + F u) / (2 eps) to leading order, which the forcing term of
    Eq. ShearEqCom cancels; without it (or with its sign flipped) the recovered S would
    carry (u F + F u) / eps over cs^2 (tau_f - A), off the diagonal too.  The traceless
    part of S must stay three orders of magnitude below that size."""
    cfg = {"nx": 4, "ny": 4, "periodic_x": 1, "periodic_y": 1, "walls": [{}] * 4,
           "tau_f": 0.9, "tau_T": 0.8, "A": 0.2, "B": 0.1, "sigma": 1.3, "Q": 0.0,
           "Da": 1e-2, "Ra": 0.0, "Pr": 1.0, "J": 1.0, "eps": 0.5, "ax": 3e-4, "ay": -2e-4,
           "T_hot": 1.0, "T_cold": 0.0, "F_eps": None, "L": 16}
    o = oracle_mod.Oracle(cfg)
    for t in (10, 60):
        o.step(t - o.time)
        f = o.fields()
        u = np.array([f["ux"][0, 0], f["uy"][0, 0]])
        o.step(1)
        f1 = o.fields()
        dudt = np.array([f1["ux"][0, 0], f1["uy"][0, 0]]) - u
        half_diff = 0.5 * (f1["Sxx"] - f1["Syy"])
        dev = max(np.abs(f1["Sxy"]).max(), np.abs(half_diff).max())
        scale = 2 * np.linalg.norm(u) * np.linalg.norm(dudt) / cfg["eps"] / (CS2 * (cfg["tau_f"] - cfg["A"]))
        assert scale > 1e-6
        assert dev < 1e-3 * scale, (t, dev, scale)
        assert np.abs(f1["ux"] - f1["ux"].mean()).max() < 1e-16
