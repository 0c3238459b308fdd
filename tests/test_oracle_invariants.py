"""Invariants, special cases and the complex-step derivative of the oracle.

  * Fully periodic box: the collision conserves sum_i f_i = rho0 per node (the EDF and
    the forcing have zero mass moment, App. A), so total mass is exact; with no force
    total momentum is exact; with a heat source the thermal energy grows by Q per node
    and step (sigma T = sum g + Q/2 and the moments of Q_i, Sec. 3.2).
  * Pure conduction between isothermal side walls: the average Nusselt number of
    Eq. AvNuss is exactly 1.
  * Complex-step derivatives of the average Nusselt number with respect to the porosity
    field agree with central finite differences of the real oracle.
  * The paper's own printed Nusselt numbers (Table Tab:Square1) as context within the
    discretization error of a coarser grid.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("seed", range(3))
def test_periodic_conservation(oracle_mod, seed):
    cfg = W.random_case(seed, 24, 20, periodic_x=1, periodic_y=1, with_Q=True)
    cfg["walls"] = [{}] * 4
    o = oracle_mod.Oracle(cfg)
    f0, g0 = o.populations(post=False)
    n = cfg["nx"] * cfg["ny"]
    for _ in range(5):
        o.step(7)
    f1, g1 = o.populations(post=False)
    assert abs(f1.sum() - n * 1.0) < 1e-11 * n
    assert abs(f0.sum() - n * 1.0) < 1e-11 * n
    assert abs((g1.sum() - g0.sum()) - 35 * n * cfg["Q"]) < 1e-11 * n


def test_periodic_momentum_without_force(oracle_mod):
    cfg = W.random_case(7, 20, 16, periodic_x=1, periodic_y=1)
    cfg.update({"walls": [{}] * 4, "Da": float("inf"), "Ra": 0.0, "ax": 0.0, "ay": 0.0,
                "F_eps": 0.0})
    o = oracle_mod.Oracle(cfg)
    cx, cy, _ = oracle_mod.lattice()
    f0, _ = o.populations(post=False)
    o.step(50)
    f1, _ = o.populations(post=False)
    for c in (cx, cy):
        m0 = np.einsum("i,iyx->", c.astype(float), f0)
        m1 = np.einsum("i,iyx->", c.astype(float), f1)
        assert abs(m1 - m0) < 1e-13


def test_conduction_cavity_nusselt_is_one(oracle_mod):
    n = 20
    cfg = W.cavity(n=n, Ra=0.0, Pr=1.0)
    cfg.update({"A": 0.2, "B": 0.1, "tau_f": 1.0, "tau_T": 1.0})
    x = np.arange(n, dtype=float)
    cfg["T_init"] = np.repeat((1.0 - x / (n - 1))[None, :], n, axis=0)
    o = oracle_mod.Oracle(cfg)
    o.step(2000)
    assert abs(o.nusselt(0) - 1.0) < 1e-12
    assert abs(o.nusselt(1) - 1.0) < 1e-12


def test_complex_step_matches_finite_difference(oracle_mod):
    """d Nu / d eps along a smooth direction: complex step (exact to round-off) vs a
    central difference of the real oracle (truncation ~h^2)."""
    n, steps = 12, 60
    cfg = W.cavity(n=n, Ra=1e5, Pr=1.0, Da=1e-2)
    rng = np.random.default_rng(3)
    eps0 = 0.6 + W.smooth_field(n, n, rng, 0.15)
    delta = W.smooth_field(n, n, rng, 1.0)

    def nu_real(e):
        c = dict(cfg, eps_field=e)
        o = oracle_mod.Oracle(c)
        o.step(steps)
        return o.nusselt(0)

    h = 1e-6
    fd = (nu_real(eps0 + h * delta) - nu_real(eps0 - h * delta)) / (2 * h)
    hc = 1e-30
    c = dict(cfg, eps_field=eps0 + 1j * hc * delta)
    oc = oracle_mod.Oracle(c, complex_step=True)
    oc.step(steps)
    nu_c = oc.nusselt(0)
    cs = nu_c.imag / hc
    assert abs(nu_c.real - nu_real(eps0)) < 1e-13
    assert abs(cs - fd) < 1e-6 * max(1.0, abs(cs))
    assert abs(cs) > 1e-6


def test_paper_table_context(oracle_mod):
    """Nusselt numbers of Table Tab:Square1 at Ra = 1e3 (eps 0.4 / 0.6 / 0.9, Da 1e-2,
    Pr 1, 120 x 120) as context: a 40 x 40 grid run to the paper's criterion lands
    within half a percent."""
    with open(os.path.join(GOLDEN, "table_square1_nusselt.json")) as fh:
        table = json.load(fh)
    for row in table["rows"]:
        if row["Ra"] != 1e3 or row["Da"] != 1e-2:
            continue
        cfg = W.cavity(n=40, eps=row["eps"], Da=row["Da"], Ra=row["Ra"], Pr=1.0)
        o = oracle_mod.Oracle(cfg)
        assert o.run_to_steady(1e-6, 200000)
        assert abs(o.nusselt(0) - row["Nu"]) < 0.005 * row["Nu"]


def test_residual_of_decaying_waves(oracle_mod):
    """The convergence residuals (Sec. 4; reading R13) on two shear waves of different
    wave numbers (u_x along y, u_y along x) and a temperature wave in a periodic box: the
    waves decay at nu_e k^2 and alpha_e k^2 / sigma, so the fields at t and t - 100 are
    known in closed form and so are both residuals.  Within 1 %: the Euclidean norm of u
    per node (a sum of |u_x| + |u_y| gives 18 % more), normalisation by the newer fields
    (the older ones give 17 % less) and T itself, not T - T0, in the L1 denominator."""
    n, cs2 = 64, 1.0 / 3.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    k1, k2 = 2 * np.pi / n, 4 * np.pi / n
    a, b, c = 1e-3, 1e-3, 0.1
    cfg = {"nx": n, "ny": n, "periodic_x": 1, "periodic_y": 1, "walls": [{}] * 4,
           "Da": float("inf"), "Ra": 0.0, "F_eps": 0.0, "tau_f": 1.0, "tau_T": 1.0,
           "A": 0.0, "B": 0.0, "eps": 1.0, "sigma": 1.0, "T_hot": 1.0, "T_cold": 0.0,
           "ux_init": a * np.sin(k1 * y), "uy_init": b * np.sin(k2 * x),
           "T_init": 0.5 + c * np.sin(k1 * x + 0.3)}
    nu = alpha = cs2 * 0.5
    o = oracle_mod.Oracle(cfg)
    t0, lag = 300, 100
    o.step(t0)
    assert o.residual() == (None, None)
    o.step(lag)
    ru, rT = o.residual()

    def exact(t):
        return (a * np.exp(-nu * k1 * k1 * t) * np.sin(k1 * y),
                b * np.exp(-nu * k2 * k2 * t) * np.sin(k2 * x),
                0.5 + c * np.exp(-alpha * k1 * k1 * t) * np.sin(k1 * x + 0.3))

    ux1, uy1, T1 = exact(t0 + lag)
    ux0, uy0, T0 = exact(t0)
    Ru = np.sum(np.hypot(ux1 - ux0, uy1 - uy0)) / np.sum(np.hypot(ux1, uy1))
    RT = np.sum(np.abs(T1 - T0)) / np.sum(np.abs(T1))
    assert abs(ru / Ru - 1) < 0.01, (ru, Ru)
    assert abs(rT / RT - 1) < 0.01, (rT, RT)
