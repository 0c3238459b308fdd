"""Pins of the whole oracle time step (bulk + boundary scheme) against closed-form or
independently computed steady solutions of the REV equations (Sec. 2), with the
second-order spatial convergence the paper reports (Sec. 4.1, Figs. AccurFig and
AccurGradFig).  Errors use the relative global error E of Sec. 4.
"""
import numpy as np
import pytest

import workloads as W
from closed_forms import (CS2, E, brinkman_profile, forchheimer_bvp, mixed_convection_cfg,
                          mixed_convection_errors, order, poiseuille_cfg)


@pytest.mark.parametrize("A", [0.1, 0.0, -0.2])
def test_brinkman_poiseuille_second_order(oracle_mod, A):
    errs_u, errs_s = [], []
    ns = (17, 33, 65)
    for ny in ns:
        cfg, c = poiseuille_cfg(ny, A, F_eps=0.0)
        o = oracle_mod.Oracle(cfg)
        assert o.run_to_steady(1e-10, 300000)
        f = o.fields()
        y = np.arange(ny, dtype=float)
        ua, dua = brinkman_profile(y, c)
        errs_u.append(E(ua, f["ux"][:, 0]))
        errs_s.append(E(dua[1:-1], f["Sxy"][1:-1, 0]))
        # the boundary scheme is not exactly mass conserving: a small wall-normal
        # velocity next to the walls is a discretization error that vanishes with ny
        assert np.abs(f["uy"]).max() < 2e-4 * np.abs(ua).max()
    assert errs_u[-1] < 2e-3 and errs_s[-1] < 5e-3
    assert order(errs_u[1], errs_u[2], ns[1], ns[2]) > 1.7
    assert order(errs_s[1], errs_s[2], ns[1], ns[2]) > 1.8


def test_brinkman_forchheimer_channel(oracle_mod):
    """Ergun F_eps: compare with an independent 1-D boundary-value solve."""
    errs = []
    ns = (33, 65)
    for ny in ns:
        cfg, c = poiseuille_cfg(ny, 0.1, F_eps=None)
        c["nu"] = CS2 * (0.8 - 0.1 - 0.5)
        Feps = 1.75 / np.sqrt(150 * c["eps"] ** 3)
        # drive at Re close to 12 so that the quadratic drag is not negligible
        cfg["ax"] *= 12.0
        c["a"] = cfg["ax"]
        o = oracle_mod.Oracle(cfg)
        assert o.run_to_steady(1e-10, 300000)
        ref, m = forchheimer_bvp(c, Feps)
        yref = np.linspace(0, c["H"], m)
        y = np.arange(ny, dtype=float)
        ua = np.interp(y, yref, ref)
        un = o.fields()["ux"][:, 0]
        errs.append(E(ua, un))
        # the quadratic drag changes the profile noticeably
        brink, _ = brinkman_profile(y, c)
        assert E(brink, ua) > 0.01
    assert errs[-1] < 2e-3
    assert order(errs[0], errs[1], ns[0], ns[1]) > 1.7


def test_brinkman_couette_second_order(oracle_mod):
    """Moving top wall, no drive: u = u0 sinh(r y) / sinh(r H), r = sqrt(eps / (J K)).
    The node next to the moving wall carries most of the error; the order reaches two
    only on the finer grids."""
    errs = []
    ns = (33, 65, 129)
    for ny in ns:
        H = ny - 1
        cfg = W.channel(ny=ny, A=0.1, B=0.1, tau=0.8, ax=0.0, F_eps=0.0, eps=0.7, Da=1e-2)
        u0 = 0.01 * 16 / H
        cfg["walls"][3]["ux"] = u0
        o = oracle_mod.Oracle(cfg)
        assert o.run_to_steady(1e-10, 300000)
        K = 1e-2 * H * H
        r = np.sqrt(0.7 / K)
        y = np.arange(ny, dtype=float)
        ua = u0 * np.sinh(r * y) / np.sinh(r * H)
        errs.append(E(ua, o.fields()["ux"][:, 0]))
    assert errs[-1] < 1.5e-3
    assert order(errs[1], errs[2], ns[1], ns[2]) > 1.75


@pytest.mark.parametrize("kind", ["dirichlet", "neumann"])
def test_conduction_is_an_exact_fixed_point(oracle_mod, kind):
    """u = 0, no buoyancy, no source: a linear temperature profile solves the discrete
    model exactly (local grad T scheme and both thermal boundary schemes are exact for
    linear fields), so T and grad T stay linear to round-off."""
    ny, slope = 24, 0.8 / 23
    cfg = W.channel(ny=ny, nx=5, ax=0.0, A=0.05, B=-0.1, tau=0.9, T_bottom=0.1, T_top=0.9)
    if kind == "neumann":
        cfg["walls"][2] = {"kind": "dTdn", "dTdn": slope}
    o = oracle_mod.Oracle(cfg)
    o.step(10000)
    f = o.fields()
    y = np.arange(ny, dtype=float)
    Tlin = 0.1 + slope * y
    assert np.abs(f["T"] - Tlin[:, None]).max() < 1e-12
    assert np.abs(f["dTdy"] - slope).max() < 1e-12
    assert np.abs(f["dTdx"]).max() < 1e-12
    assert np.abs(f["ux"]).max() < 1e-14 and np.abs(f["uy"]).max() < 1e-14


def _mixed_convection(oracle_mod, ny, tau):
    cfg, steps, exact = mixed_convection_cfg(ny, tau)
    o = oracle_mod.Oracle(cfg)
    o.step(steps)
    return mixed_convection_errors(o.fields(), exact)


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_mixed_convection_channel_second_order(oracle_mod, tau):
    """Closed forms for u_x, T, du_x/dy, dT/dy, each converging at second order; as in
    the Couette case the velocity next to the moving wall approaches order two from
    below on these grids."""
    ns = (17, 33, 65)
    res = [_mixed_convection(oracle_mod, n, tau) for n in ns]
    for k, lo in zip(range(4), (1.5, 1.75, 1.75, 1.75)):
        e1, e2 = res[1][k], res[2][k]
        assert e2 < 1e-2, (k, res)
        assert order(e1, e2, ns[1], ns[2]) > lo, (k, res)
        assert order(res[0][k], e1, ns[0], ns[1]) < order(e1, e2, ns[1], ns[2]) + 0.3
    assert res[-1][4] < 1e-3


def test_adiabatic_wall_nodes_take_the_prescribed_gradient(oracle_mod):
    """Reading R5 (Sec. 3.4: on a prescribed-gradient wall grad T(x_b) is the known one): in a
    convecting cavity the adiabatic wall nodes report and collide with dT/dy = 0 exactly,
    while the next node inward carries a nonzero gradient.  Recomputing the wall node's
    gradient from its rebuilt populations would give tau_T / (tau_T - B) times that of x_f."""
    cfg = W.cavity(n=24, eps=0.6, Da=1e-2, Ra=1e4, Pr=1.0)
    o = oracle_mod.Oracle(cfg)
    o.step(3000)
    f = o.fields()
    inner = slice(1, -1)                 # the corners belong to the isothermal walls (R8)
    assert np.abs(f["dTdy"][0, inner]).max() == 0.0
    assert np.abs(f["dTdy"][-1, inner]).max() == 0.0
    assert np.abs(f["dTdy"][1, inner]).max() > 1e-4
    assert np.abs(f["dTdy"][-2, inner]).max() > 1e-4
