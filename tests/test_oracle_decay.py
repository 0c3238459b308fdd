"""Pins of the transport coefficients the oracle realises.

The Chapman-Enskog analysis fixes the effective viscosity nu_e = cs^2 (tau_f - A - 1/2)
(Sec. 3.1; App. A) and the effective diffusivity alpha_e = sigma cs^2 (tau_T - B - 1/2)
(Eq. Therdiff) of the recovered equations (Eq. GoverneEq).  A shear wave and a
temperature wave in a periodic box decay at nu_e k^2 and alpha_e k^2 / sigma; a
temperature wave carried by a uniform stream moves at u / sigma.  The measured rates
must approach these values at second order in k.
"""
import numpy as np
import pytest

CS2 = 1.0 / 3.0


def _box(n, tau_f, tau_T, A, B, eps=1.0, sigma=1.0, **kw):
    cfg = {"nx": kw.pop("nx", 4), "ny": n, "periodic_x": 1, "periodic_y": 1,
           "walls": [{}] * 4, "Da": float("inf"), "Ra": 0.0, "F_eps": 0.0,
           "tau_f": tau_f, "tau_T": tau_T, "A": A, "B": B, "eps": eps, "sigma": sigma,
           "T_hot": 1.0, "T_cold": 0.0}
    cfg.update(kw)
    return cfg


def _shear_rate(oracle_mod, n, tau, A, eps):
    y = np.arange(n, dtype=float)
    k = 2 * np.pi / n
    U = 1e-3
    cfg = _box(n, tau, tau, A, 0.0, eps=eps)
    cfg["ux_init"] = np.repeat((U * np.sin(k * y))[:, None], 4, axis=1)
    o = oracle_mod.Oracle(cfg)
    nu_e = CS2 * (tau - A - 0.5)
    t1 = int(0.1 / (nu_e * k * k))
    t2 = int(0.6 / (nu_e * k * k))
    o.step(t1)
    a1 = 2 / n * (o.fields()["ux"][:, 0] * np.sin(k * y)).sum()
    o.step(t2 - t1)
    a2 = 2 / n * (o.fields()["ux"][:, 0] * np.sin(k * y)).sum()
    return np.log(a1 / a2) / (t2 - t1) / (nu_e * k * k)


@pytest.mark.parametrize("tau,A", [(1.0, 0.3), (1.0, 0.0), (1.0, -0.2), (0.8, 0.25), (0.6, 0.0)])
def test_shear_wave_viscosity(oracle_mod, tau, A):
    r32 = _shear_rate(oracle_mod, 32, tau, A, eps=0.7)
    r64 = _shear_rate(oracle_mod, 64, tau, A, eps=0.7)
    assert abs(r64 - 1) < 2e-3
    assert abs(r64 - 1) < 0.35 * abs(r32 - 1) + 1e-6


def _thermal_wave(oracle_mod, n, tau, B, sigma, eps, U):
    """Returns (decay-rate ratio, phase-speed ratio) of a temperature wave in x."""
    x = np.arange(n, dtype=float)
    k = 2 * np.pi / n
    cfg = _box(4, 1.0, tau, 0.0, B, eps=eps, sigma=sigma, nx=n)
    cfg["T_init"] = np.repeat((0.5 + 0.1 * np.sin(k * x))[None, :], 4, axis=0)
    cfg["ux_init"] = np.full((4, n), U)
    o = oracle_mod.Oracle(cfg)
    alpha = sigma * CS2 * (tau - B - 0.5)
    t1 = int(0.1 / (alpha / sigma * k * k))
    t2 = int(0.6 / (alpha / sigma * k * k))
    o.step(t1)
    c1 = ((o.fields()["T"][0] - 0.5) * np.exp(-1j * k * x)).sum()
    o.step(t2 - t1)
    c2 = ((o.fields()["T"][0] - 0.5) * np.exp(-1j * k * x)).sum()
    rate = np.log(abs(c1) / abs(c2)) / (t2 - t1) / (alpha / sigma * k * k)
    dphi = -np.angle(c2 / c1)
    speed = dphi / k / (t2 - t1) / (U / sigma) if U != 0 else 0.0
    return rate, speed


@pytest.mark.parametrize("tau,B,sigma", [(1.0, 0.3, 1.0), (1.0, -0.2, 1.0), (0.8, 0.1, 1.3),
                                         (1.0, 0.0, 1.0)])
def test_thermal_wave_diffusivity(oracle_mod, tau, B, sigma):
    r32, _ = _thermal_wave(oracle_mod, 32, tau, B, sigma, 0.6, 0.0)
    r64, _ = _thermal_wave(oracle_mod, 64, tau, B, sigma, 0.6, 0.0)
    assert abs(r64 - 1) < 2e-3
    assert abs(r64 - 1) < 0.35 * abs(r32 - 1) + 1e-6


@pytest.mark.parametrize("sigma,eps", [(1.0, 0.5), (1.3, 0.7), (1.0, 1.0)])
def test_advected_thermal_wave(oracle_mod, sigma, eps):
    """Uniform stream with eps != sigma: exercises the u u terms of <M> and P_i."""
    r64, s64 = _thermal_wave(oracle_mod, 64, 1.0, 0.2, sigma, eps, 0.02)
    r32, s32 = _thermal_wave(oracle_mod, 32, 1.0, 0.2, sigma, eps, 0.02)
    assert abs(r64 - 1) < 5e-3 and abs(s64 - 1) < 2e-3
    assert abs(r64 - 1) < 0.4 * abs(r32 - 1) + 1e-4
