"""Pins of the 3-D (D3Q19) oracle's single-node arithmetic against what the paper fixes.

As for the 2-D lattice, each check compares the oracle with a fact the paper or the
mathematics states, not with a retyping of the oracle's own formula:
  * the velocity moments of the equilibria, the forcing and the thermal sources that the
    Chapman-Enskog analysis requires (App. A moment lists; Sec. 3.2), on random states
    with eps != sigma and sigma != 1, so that the (1/eps - 1/sigma) u u part of P_i
    (Eq. Eq:Tforce) is fixed by its first moment;
  * the closed forms of s_0 and F_0 (App. A, last equation) with the rest weight 1/3;
  * the implicit definition of the velocity through the quadratic drag (Sec. 3.1);
  * recovery of a prescribed 3 x 3 shear rate from the non-equilibrium second moment
    (Eq. ShearEqCom);
  * recovery of grad T from a prescribed first moment (Eqs. SonaT, MatrM, MatrN) along
    and across u with eps != sigma: across u the divisor is cs^2 sigma (B - tau_T)
    - eps p / (2 rho0); along u it also loses (1/eps - 1/sigma) |u|^2 / 2, the second
    factor of Eq. detMatr (a sign slip in the u u part of <M> changes it);
  * the conservation of mass and the momentum and energy balance of one collision.
"""
import numpy as np
import pytest

import oracle.oracle3 as O3

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def lat():
    c, w = O3.lattice()
    return c.astype(np.float64), w


def _cfg(rng, **kw):
    cfg = {"nx": 6, "ny": 6, "nz": 6, "periodic_x": 1, "periodic_y": 1, "periodic_z": 1,
           "walls": [{}, {}], "tau_f": rng.uniform(0.6, 1.5), "tau_T": rng.uniform(0.6, 1.5),
           "A": rng.uniform(-0.2, 0.05), "B": rng.uniform(-0.2, 0.05),
           "sigma": rng.uniform(0.7, 1.6), "Q": rng.uniform(-1e-3, 1e-3),
           "Da": 10 ** rng.uniform(-3, -1), "Ra": 1e4, "Pr": 1.0, "J": 1.0, "Ma": 0.1,
           "eps": rng.uniform(0.3, 1.0), "a": (0.0, 0.0, 0.0), "T_hot": 1.0, "T_cold": 0.0,
           "F_eps": None}
    cfg.update(kw)
    return cfg


def _moments(c):
    m0 = lambda x: x.sum()
    m1 = lambda x: np.einsum("i,ia->a", x, c)
    m2 = lambda x: np.einsum("i,ia,ib->ab", x, c, c)
    m3 = lambda x: np.einsum("i,ia,ib,ic->abc", x, c, c, c)
    return m0, m1, m2, m3


def _delta_u(u):
    I = np.eye(3)
    return np.einsum("a,bc->abc", u, I) + np.einsum("b,ac->abc", u, I) + np.einsum("c,ab->abc", u, I)


@pytest.mark.parametrize("seed", range(20))
def test_moment_identities(lat, seed):
    c, w = lat
    rng = np.random.default_rng(seed)
    cfg = _cfg(rng)
    d = O3.derived(cfg)
    eps, T = cfg["eps"], rng.uniform(0.0, 2.0)
    u = rng.uniform(-0.1, 0.1, 3)
    p = rng.uniform(-0.01, 0.01)
    S = rng.uniform(-0.01, 0.01, (3, 3))
    S = S + S.T                      # symmetric, with a trace
    gT = rng.uniform(-0.05, 0.05, 3)
    F = rng.uniform(-1e-3, 1e-3, 3)
    t = O3.node_terms(cfg, eps, T, u, p, S, gT, F)
    rho0, sig, tf, tT, Q = 1.0, cfg["sigma"], cfg["tau_f"], cfg["tau_T"], cfg["Q"]
    A, B = d["A"], d["B"]
    I = np.eye(3)
    m0, m1, m2, m3 = _moments(c)
    tol = 1e-15
    # flow equilibrium (App. A: moments of f^{e(0)} and of the shear-rate part)
    fe0, r = t["feq0"], t["r"]
    assert abs(m0(fe0) - rho0) < tol
    assert np.allclose(m1(fe0), rho0 * u, atol=tol)
    assert np.allclose(m2(fe0), eps * p * I + rho0 * np.outer(u, u) / eps, atol=tol)
    assert np.allclose(m3(fe0), CS2 * rho0 * _delta_u(u), atol=tol)
    assert abs(m0(r)) < tol and np.allclose(m1(r), 0, atol=tol)
    assert np.allclose(m2(rho0 * r), CS2 * rho0 * A * S, atol=tol)
    # closed forms of s_0 (through f_0^{e(0)}) and F_0 with the rest weight 1/3
    assert abs(w[0] - 1.0 / 3.0) < 1e-16
    s0 = -w[0] / (2 * eps * CS2) * (u @ u)
    assert abs(fe0[0] - (rho0 - (1 - w[0]) * eps * p / CS2 + rho0 * s0)) < tol
    F0 = -w[0] * (1 - 1 / (2 * tf)) * (u @ F) / (eps * CS2)
    assert abs(t["F"][0] - F0) < tol
    # forcing term (App. A: moments of F_i)
    Fi = t["F"]
    assert abs(m0(Fi)) < tol
    assert np.allclose(m1(Fi), (1 - 1 / (2 * tf)) * rho0 * F, atol=tol)
    assert np.allclose(m2(Fi), (1 - 1 / (2 * tf)) * rho0 * (np.outer(u, F) + np.outer(F, u)) / eps, atol=tol)
    # temperature equilibrium (Sec. 3.2 moment list)
    ge0, gB = t["geq0"], t["gB"]
    assert abs(m0(ge0) - sig * T) < tol
    assert np.allclose(m1(ge0), T * u, atol=tol)
    assert np.allclose(m2(ge0), T * np.outer(u, u) / eps + CS2 * sig * T * I + eps * p * T / rho0 * I, atol=tol)
    assert np.allclose(m3(ge0), CS2 * T * _delta_u(u), atol=tol)
    assert abs(m0(gB)) < tol
    assert np.allclose(m1(gB), sig * CS2 * B * gT, atol=tol)
    assert np.allclose(m2(gB), 0, atol=tol)
    # thermal sources: the first moment of P_i carries the (1/eps - 1/sigma) u (u . grad T) term
    P, Qi = t["P"], t["Q"]
    assert abs(m0(P)) < tol
    assert np.allclose(m1(P), (1 - 1 / (2 * tT)) * (T * F + eps * p * gT / rho0
                                                   + (1 / eps - 1 / sig) * u * (u @ gT)), atol=tol)
    assert np.allclose(m2(P), 0, atol=tol)
    assert abs(m0(Qi) - (1 - 1 / (2 * tT)) * Q) < tol
    assert np.allclose(m1(Qi), (1 - 1 / (2 * tT)) * u * Q / sig, atol=tol)


def _drag_F(cfg, d, eps, u, G):
    """Total force of Eq. ForceEq with the Ergun F_eps."""
    Feps = 1.75 / np.sqrt(150 * eps ** 3)
    return -eps * d["nu"] / d["K"] * u - eps * Feps / np.sqrt(d["K"]) * np.linalg.norm(u) * u + eps * G


@pytest.mark.parametrize("seed", range(10))
def test_drag_solve_satisfies_implicit_definition(lat, seed):
    """u = sum c f / rho0 + F(u) / 2 with F quadratic in u (Sec. 3.1): populations built with
    the first moment a chosen u requires return that u and its force."""
    c, w = lat
    rng = np.random.default_rng(100 + seed)
    G = rng.uniform(-1e-4, 1e-4, 3)
    cfg = _cfg(rng, Q=0.0, Ra=0.0, A=0.0, B=0.0, a=tuple(G))
    d = O3.derived(cfg)
    eps = cfg["eps"]
    u = rng.uniform(-0.08, 0.08, 3)
    j = u - 0.5 * _drag_F(cfg, d, eps, u, G)          # the required sum_i c_i f_i
    f = w * (1 + rng.uniform(-0.05, 0.05, 19))
    f = f + w * (c @ (j - c.T @ f)) / CS2            # fix the first moment to j
    g = w * 0.5
    m = O3.node_macro(cfg, eps, f, g)
    assert np.abs(m["u"] - u).max() < 1e-15
    assert np.abs(m["F"] - _drag_F(cfg, d, eps, u, G)).max() < 1e-16


def _base_state(cfg, eps, p, u, T):
    t = O3.node_terms(cfg, eps, T, u, p, np.zeros(9), np.zeros(3), np.zeros(3))
    return t["feq0"], t["geq0"]


@pytest.mark.parametrize("seed", range(10))
def test_shear_rate_from_nonequilibrium_part(lat, seed):
    """With no force, S = sum c c (f - f^{e(0)}) / (cs^2 rho0 (A - tau_f)) (Eq. ShearEqCom): a
    state f^{e(0)} + Delta whose Delta has a prescribed traceless second moment returns the
    prescribed 3 x 3 S and leaves p, u and T unchanged."""
    c, w = lat
    rng = np.random.default_rng(200 + seed)
    cfg = _cfg(rng, Da=float("inf"), Q=0.0, Ra=0.0, F_eps=0.0)
    d = O3.derived(cfg)
    eps, p, T = cfg["eps"], rng.uniform(-0.01, 0.01), rng.uniform(0, 1)
    u = rng.uniform(-0.05, 0.05, 3)
    St = rng.uniform(-0.01, 0.01, (3, 3))
    St = St + St.T
    St -= np.trace(St) / 3 * np.eye(3)
    X = CS2 * (d["A"] - cfg["tau_f"]) * St
    # the second-moment-only perturbation of D3Q19: omega_i (c.X.c - cs^2 tr X) / (2 cs^4)
    delta = w * (np.einsum("ab,ia,ib->i", X, c, c) - CS2 * np.trace(X)) / (2 * CS2 ** 2)
    assert abs(delta.sum()) < 1e-17 and np.abs(c.T @ delta).max() < 1e-17
    f0, g0 = _base_state(cfg, eps, p, u, T)
    m = O3.node_macro(cfg, eps, f0 + delta, g0)
    assert np.abs(m["S"] - St).max() < 1e-14
    assert abs(m["p"] - p) < 1e-15 and np.abs(m["u"] - u).max() < 1e-15 and abs(m["T"] - T) < 1e-15


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("orient", ["perp", "par"])
def test_temperature_gradient_eigendirections(lat, seed, orient):
    """grad T from <M> grad T = <N> (Eqs. SonaT, MatrM, MatrN) with eps != sigma: for N
    across u the divisor is cs^2 sigma (B - tau_T) - eps p / (2 rho0); along u it also
    loses (1/eps - 1/sigma) |u|^2 / 2 (the second factor of Eq. detMatr)."""
    c, w = lat
    rng = np.random.default_rng(300 + seed)
    cfg = _cfg(rng, Da=float("inf"), Q=0.0, Ra=0.0, F_eps=0.0, eps=rng.uniform(0.3, 0.6),
               sigma=rng.uniform(1.1, 1.6))
    d = O3.derived(cfg)
    eps, sig, p, T = cfg["eps"], cfg["sigma"], rng.uniform(-0.01, 0.01), rng.uniform(0, 1)
    u = rng.uniform(-0.15, 0.15, 3)
    uhat = u / np.linalg.norm(u)
    if orient == "perp":
        v = rng.normal(size=3)
        dirv = v - (v @ uhat) * uhat
        dirv /= np.linalg.norm(dirv)
    else:
        dirv = uhat
    N = rng.uniform(0.5, 2.0) * 1e-3 * dirv
    dg = w * (c @ N) / CS2                  # sum dg = 0, sum c dg = N, sum c c dg = 0
    f0, g0 = _base_state(cfg, eps, p, u, T)
    m = O3.node_macro(cfg, eps, f0, g0 + dg)
    a = CS2 * sig * (d["B"] - cfg["tau_T"]) - eps * p / 2
    if orient == "par":
        a -= 0.5 * (1 / eps - 1 / sig) * (u @ u)
    # N is a difference of O(T omega) populations: rounding of about 1e-16 T / abs(N) relative
    assert np.allclose(m["dT"], N / a, rtol=2e-12, atol=1e-17)
    assert abs(m["T"] - T) < 1e-15
    # along u the two divisors differ by more than the tolerance
    assert 0.5 * (1 / eps - 1 / sig) * (u @ u) > 1e-4 * abs(a)


@pytest.mark.parametrize("seed", range(10))
def test_collision_conserves_mass_and_balances_energy(lat, seed):
    """sum f* = sum f - (sum f - rho0) / tau_f, sum c f* = rho0 (u + F/2) and
    sum g* = sigma T + Q/2 follow from the moment lists and sigma T = sum g + Q/2 (Sec. 3.2)."""
    c, w = lat
    rng = np.random.default_rng(400 + seed)
    cfg = _cfg(rng, a=tuple(rng.uniform(-1e-4, 1e-4, 3)))
    eps = cfg["eps"]
    f = w * (1 + rng.uniform(-0.05, 0.05, 19))
    f[0] = 1.0 - f[1:].sum() + rng.uniform(-1e-3, 1e-3)
    g = w * (0.5 + rng.uniform(-0.05, 0.05, 19))
    m = O3.node_macro(cfg, eps, f, g)
    fo, go = O3.node_collide(cfg, eps, f, g)
    tf = cfg["tau_f"]
    assert abs(fo.sum() - (f.sum() - (f.sum() - 1.0) / tf)) < 1e-15
    assert np.allclose(c.T @ fo, m["u"] + 0.5 * m["F"], atol=1e-15)
    assert abs(go.sum() - (cfg["sigma"] * m["T"] + 0.5 * cfg["Q"])) < 1e-15


def test_uniformly_accelerating_flow_has_no_shear():
    """A porous flow that is uniform in space and accelerates under a body force in an
    oblique direction (Darcy and Forchheimer drag on) has no velocity gradient.  The
    non-equilibrium second moment of such a state is -(u F + F u) / (2 eps) to leading
    order, which the forcing term of Eq. ShearEqCom cancels; without that cancellation
    (or with its sign flipped) the recovered S would carry (u F + F u) / eps over
    cs^2 (tau_f - A), off the diagonal too.  The traceless part of S must stay at least
    three orders of magnitude below that size."""
    cfg = {"nx": 4, "ny": 4, "nz": 4, "periodic_x": 1, "periodic_y": 1, "periodic_z": 1,
           "walls": [{}, {}], "tau_f": 0.9, "tau_T": 0.8, "A": 0.2, "B": 0.1, "sigma": 1.3, "Q": 0.0,
           "Da": 1e-2, "Ra": 0.0, "Pr": 1.0, "J": 1.0, "Ma": 0.1, "eps": 0.5, "a": (3e-4, -2e-4, 1e-4),
           "T_hot": 1.0, "T_cold": 0.0, "F_eps": None, "L": 16}
    o = O3.Oracle3(cfg)
    for t in (10, 60):
        o.step(t - o.time)
        f = o.fields()
        u = np.array([f[k][0, 0, 0] for k in ("ux", "uy", "uz")])
        o.step(1)
        f1 = o.fields()
        dudt = np.array([f1[k][0, 0, 0] for k in ("ux", "uy", "uz")]) - u
        comps = ("Sxx", "Sxy", "Sxz", "Syy", "Syz", "Szz")
        Sv = {k: f1[k] for k in comps}
        tr = (Sv["Sxx"] + Sv["Syy"] + Sv["Szz"]) / 3
        dev = max(np.abs(Sv["Sxy"]).max(), np.abs(Sv["Sxz"]).max(), np.abs(Sv["Syz"]).max(),
                  *(np.abs(Sv[k] - tr).max() for k in ("Sxx", "Syy", "Szz")))
        scale = 2 * np.linalg.norm(u) * np.linalg.norm(dudt) / cfg["eps"] / (CS2 * (cfg["tau_f"] - cfg["A"]))
        assert scale > 1e-6
        assert dev < 1e-3 * scale, (t, dev, scale)
        # and the flow stays uniform
        assert np.abs(f1["ux"] - f1["ux"].mean()).max() < 1e-16
