"""Closed-form and independently computed steady solutions of the REV equations (Sec. 2)
for the channel flows of Sec. 4.1, shared by the oracle pins and the GPU flow tests.
Errors use the relative global error E of Sec. 4."""
import numpy as np
from scipy.linalg import solve_banded

import workloads as W

CS2 = 1.0 / 3.0


def E(a, n):
    return np.abs(a - n).sum() / np.abs(a).sum()


def order(e_coarse, e_fine, n_coarse, n_fine):
    return np.log(e_coarse / e_fine) / np.log((n_fine - 1) / (n_coarse - 1))


def poiseuille_cfg(ny, A, F_eps):
    """Porous plane Poiseuille: eps 0.5, Da 1e-2, tau 0.8, Re = 1 (drive from the
    Brinkman closed form so that the centreline speed is Re nu / H)."""
    eps, Da, tau, J = 0.5, 1e-2, 0.8, 1.0
    H = ny - 1
    nu = CS2 * (tau - A - 0.5)
    K = Da * H * H
    r = np.sqrt(eps / (J * K))
    a = (nu / H) * nu / (K * (1 - 1 / np.cosh(r * H / 2)))
    cfg = W.channel(ny=ny, A=A, B=A, tau=tau, ax=a, F_eps=F_eps, eps=eps, Da=Da)
    return cfg, dict(H=H, nu=nu, K=K, r=r, a=a, eps=eps)


def brinkman_profile(y, c):
    """Steady Brinkman flow between fixed walls (Sec. 2 momentum eq. with F_eps = 0):
    nu_e u'' - (eps nu / K) u + eps a = 0, u(0) = u(H) = 0."""
    H, a, K, nu, r = c["H"], c["a"], c["K"], c["nu"], c["r"]
    u = a * K / nu * (1 - np.cosh(r * (y - H / 2)) / np.cosh(r * H / 2))
    du = -a * K / nu * r * np.sinh(r * (y - H / 2)) / np.cosh(r * H / 2)
    return u, du


def forchheimer_bvp(c, Feps, npts=20001):
    """Independent Newton finite-difference solve of
    nu_e u'' - (eps nu/K) u - (eps F_eps/sqrt K) |u| u + eps a = 0, u(0) = u(H) = 0,
    then Richardson extrapolation from npts and (npts + 1) / 2 points."""
    def solve(n):
        H, eps, K, nu, a = c["H"], c["eps"], c["K"], c["nu"], c["a"]
        h = H / (n - 1)
        u = np.zeros(n)
        for _ in range(50):
            ui = u[1:-1]
            lap = (u[:-2] - 2 * ui + u[2:]) / h ** 2
            R = nu * lap - eps * nu / K * ui - eps * Feps / np.sqrt(K) * np.abs(ui) * ui + eps * a
            diag = -2 * nu / h ** 2 - eps * nu / K - 2 * eps * Feps / np.sqrt(K) * np.abs(ui)
            off = np.full(n - 3, nu / h ** 2)
            ab = np.zeros((3, n - 2))
            ab[0, 1:] = off
            ab[1] = diag
            ab[2, :-1] = off
            du = solve_banded((1, 1), ab, -R)
            u[1:-1] += du
            if np.abs(du).max() < 1e-17:
                break
        return u
    fine = solve(npts)
    coarse = solve((npts + 1) // 2)
    return (4 * fine[::2] - coarse) / 3, (npts + 1) // 2



def mixed_convection_cfg(ny, tau, Re=5.0, A=None):
    """Sec. 4.1: porous channel with a moving hot top wall and injection through the
    walls; eps 0.6, Ra 100, Pr 1, Da 0.01, F_eps = 0, u0 = v0.  Returns (cfg, steps,
    exact) with exact = (u_x, T, du_x/dy, dT/dy, v0) on the nodes.

    The boundary scheme does not balance the normal mass flux exactly, so the pressure
    level drifts slowly (at a rate that falls roughly 15-fold per grid doubling) and the
    residual never settles to round-off; the run therefore stops at a fixed diffusive
    time 3 H^2 / nu, after which the slowest transient has decayed by e^-30.

    With A given (the accuracy study at fixed tau, Sec. 4.1), B = A, the viscosity is
    cs^2 (tau - A - 1/2) and the injection speed v0 = Re nu / H keeps Re."""
    H = ny - 1
    eps, Da, Pr, J = 0.6, 1e-2, 1.0, 1.0
    if A is None:
        v0 = 0.01 * 32.0 / H
        nu = H * v0 / Re
        A = tau - 0.5 - nu / CS2
    else:
        nu = CS2 * (tau - A - 0.5)
        v0 = Re * nu / H
    u0 = v0
    B = tau - 0.5 - nu / Pr / CS2
    K = Da * H * H
    cfg = W.channel(ny=ny, A=A, B=B, tau=tau, eps=eps, Da=Da, F_eps=0.0, ax=0.0,
                    T_bottom=0.0, T_top=1.0)
    cfg["walls"][2].update({"ux": 0.0, "uy": v0})
    cfg["walls"][3].update({"ux": u0, "uy": v0})
    cfg["ay"] = nu / K * v0          # balances the Darcy drag on the injected flow
    cfg["Ra"], cfg["Pr"] = 100.0, Pr
    z1 = Re / (2 * eps * J)
    z2 = np.sqrt(Re ** 2 + 4 * eps ** 3 * J / Da) / (2 * eps * J)
    eta = np.arange(ny) / H
    # the closed forms with the growing exponentials factored out (no overflow at large Re)
    grow = np.exp((z1 + z2) * (eta - 1)) / (1 - np.exp(-2 * z2))
    ua = u0 * grow * (1 - np.exp(-2 * z2 * eta))
    dua = u0 * grow * (z1 * (1 - np.exp(-2 * z2 * eta)) + z2 * (1 + np.exp(-2 * z2 * eta))) / H
    Pe = Pr * Re
    Ta = (np.exp(Pe * (eta - 1)) - np.exp(-Pe)) / (1 - np.exp(-Pe))
    dTa = Pe / H * np.exp(Pe * (eta - 1)) / (1 - np.exp(-Pe))
    return cfg, int(3 * H * H / nu), (ua, Ta, dua, dTa, v0)


def mixed_convection_errors(f, exact):
    """E of u_x, T, du_x/dy (= Sxy), dT/dy on the column x = 0, and max |u_y - v0| / v0."""
    ua, Ta, dua, dTa, v0 = exact
    inner = slice(1, -1)
    return (E(ua, f["ux"][:, 0]), E(Ta, f["T"][:, 0]),
            E(dua[inner], f["Sxy"][inner, 0]), E(dTa[inner], f["dTdy"][inner, 0]),
            np.abs(f["uy"][:, 0] - v0).max() / v0)
