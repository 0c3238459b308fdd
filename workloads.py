"""Seeded synthetic inputs shared by the oracle side and the GPU side of every test and
benchmark.

This module holds problem descriptions (plain dictionaries of physical parameters) and
seeded random fields only.  It contains none of the method's arithmetic: the mapping
from (Da, Ra, Pr, Ma, ...) to lattice constants, the equilibria and every step of the
time update live separately in the oracle and in the GPU library.

A problem dictionary has the keys below (all optional except nx, ny):

    nx, ny                 nodes, wall nodes included
    periodic_x, periodic_y 1 = periodic direction, 0 = a wall node at each end
    walls                  4 dicts for x-, x+, y-, y+:  {"ux", "uy", "kind", "T", "dTdn"}
                           kind "T" = isothermal at T, "dTdn" = prescribed inward normal
                           derivative of T
    L                      characteristic length (0 or absent = from the grid)
    Da, Ra, Pr, J, Ma, sigma, Q, tau_f, tau_T
    A, B                   None = from Ma, Ra, Pr; numbers = used as given
    eps                    uniform porosity;  eps_field = [ny, nx] array (optional)
    ax, ay                 external acceleration
    T_hot, T_cold          reference temperatures (T0 is their mean, dT their difference)
    F_eps                  None = Ergun relation; number = used as given (0: no Forchheimer)
    T_init, p_init, ux_init, uy_init   optional [ny, nx] initial fields
    storage                "f64" | "f32" | "f16" (GPU only)
"""
from __future__ import annotations

import numpy as np


def _cavity_walls(T_hot=1.0, T_cold=0.0):
    return [
        {"kind": "T", "T": T_hot},
        {"kind": "T", "T": T_cold},
        {"kind": "dTdn", "dTdn": 0.0},
        {"kind": "dTdn", "dTdn": 0.0},
    ]


def cavity_T_init(nx, ny, seed=0, amp=1e-3, T_hot=1.0, T_cold=0.0):
    """Mid temperature plus uniform noise of +-amp; isothermal side columns at wall T."""
    rng = np.random.default_rng(seed)
    T = 0.5 * (T_hot + T_cold) + rng.uniform(-amp, amp, size=(ny, nx))
    T[:, 0] = T_hot
    T[:, -1] = T_cold
    return T


def cavity(n=128, eps=0.6, Da=1e-2, Ra=1e5, Pr=1.0, seed=0, storage="f64", nx=None, ny=None,
           tau=1.0, Ma=0.1):
    """Natural convection in a square porous cavity: hot left wall, cold right wall,
    adiabatic top and bottom, zero velocity on all walls."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    return {
        "nx": nx, "ny": ny, "periodic_x": 0, "periodic_y": 0,
        "walls": _cavity_walls(),
        "Da": Da, "Ra": Ra, "Pr": Pr, "J": 1.0, "Ma": Ma, "sigma": 1.0, "Q": 0.0,
        "tau_f": tau, "tau_T": tau, "A": None, "B": None,
        "eps": eps, "ax": 0.0, "ay": 0.0, "T_hot": 1.0, "T_cold": 0.0, "F_eps": None,
        "T_init": cavity_T_init(nx, ny, seed),
        "storage": storage,
    }


def channel(ny=64, nx=4, eps=0.5, Da=1e-2, tau=0.8, A=0.1, B=0.1, ax=1.887e-6, F_eps=None,
            storage="f64", T_bottom=0.0, T_top=1.0, linear_T=True):
    """Force-driven porous plane channel, periodic in x, walls at y = 0 and y = ny - 1
    held at T_bottom and T_top.  The default drive gives Re close to 1 for the default
    parameters."""
    T_init = None
    if linear_T:
        y = np.arange(ny, dtype=np.float64)
        T_init = np.repeat((T_bottom + (T_top - T_bottom) * y / (ny - 1))[:, None], nx, axis=1)
    return {
        "nx": nx, "ny": ny, "periodic_x": 1, "periodic_y": 0,
        "walls": [{}, {}, {"kind": "T", "T": T_bottom}, {"kind": "T", "T": T_top}],
        "L": float(ny - 1),
        "Da": Da, "Ra": 0.0, "Pr": 1.0, "J": 1.0, "Ma": 0.1, "sigma": 1.0, "Q": 0.0,
        "tau_f": tau, "tau_T": tau, "A": A, "B": B,
        "eps": eps, "ax": ax, "ay": 0.0, "T_hot": T_top, "T_cold": T_bottom, "F_eps": F_eps,
        "T_init": T_init,
        "storage": storage,
    }


def large_cavity(n=4096, storage="f32", seed=0):
    """Throughput workload: 4096 x 4096 porous cavity, eps 0.4, Da 1e-4, Ra 1e7, Pr 0.71."""
    return cavity(n=n, eps=0.4, Da=1e-4, Ra=1e7, Pr=0.71, seed=seed, storage=storage)


def smooth_field(nx, ny, rng, amp, modes=4, kmax=3):
    """Sum of a few random low Fourier modes, scaled to max |value| = amp."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    out = np.zeros((ny, nx))
    for _ in range(modes):
        kx, ky = rng.integers(-kmax, kmax + 1, size=2)
        ph = rng.uniform(0, 2 * np.pi)
        out += rng.normal() * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
    m = np.max(np.abs(out))
    return out * (amp / m if m > 0 else 0.0)


def random_case(seed, nx, ny, periodic_x=0, periodic_y=0, storage="f64", eps_field=False,
                moving_walls=False, with_Q=False, flow_amp=0.03):
    """A randomised problem with a non-trivial initial flow, pressure and temperature, for
    element-wise parity checks.  The characteristic length is fixed at 200 lattice units
    (independent of the small grid) and Ra drawn in [1e2, 1e3], so that the buoyancy
    velocity scale stays below about 0.03 on any grid."""
    rng = np.random.default_rng(seed)
    walls = []
    for k in range(4):
        kind = "T" if rng.uniform() < 0.5 else "dTdn"
        w = {"kind": kind, "T": float(rng.uniform(0, 1)), "dTdn": float(rng.uniform(-0.01, 0.01))}
        if moving_walls:
            w["ux"] = float(rng.uniform(-0.02, 0.02))
            w["uy"] = float(rng.uniform(-0.005, 0.005))
        walls.append(w)
    cfg = {
        "nx": nx, "ny": ny, "periodic_x": periodic_x, "periodic_y": periodic_y,
        "walls": walls, "L": 200.0,
        "Da": float(10 ** rng.uniform(-3, -1)), "Ra": float(10 ** rng.uniform(2, 3)),
        "Pr": float(rng.uniform(0.7, 2.0)), "J": float(rng.uniform(0.8, 1.2)), "Ma": 0.1,
        "sigma": float(rng.uniform(0.9, 1.2)),
        "Q": float(rng.uniform(-1e-5, 1e-5)) if with_Q else 0.0,
        "tau_f": float(rng.uniform(0.7, 1.2)), "tau_T": float(rng.uniform(0.7, 1.2)),
        "A": float(rng.uniform(-0.2, 0.15)), "B": float(rng.uniform(-0.2, 0.15)),
        "eps": float(rng.uniform(0.4, 0.95)),
        "ax": float(rng.uniform(-1e-5, 1e-5)), "ay": float(rng.uniform(-1e-5, 1e-5)),
        "T_hot": 1.0, "T_cold": 0.0, "F_eps": None,
        "T_init": 0.5 + smooth_field(nx, ny, rng, 0.4),
        "p_init": smooth_field(nx, ny, rng, 2e-3),
        "ux_init": smooth_field(nx, ny, rng, flow_amp),
        "uy_init": smooth_field(nx, ny, rng, flow_amp),
        "storage": storage,
    }
    if eps_field:
        cfg["eps_field"] = 0.65 + smooth_field(nx, ny, rng, 0.25)
    return cfg


def porosity_field(n=256, seed=0, modes=16, kmax=8):
    """eps(x, y) = 0.6 + 0.2 tanh(phi), phi a sum of `modes` random Fourier modes with
    integer wave vectors 1 <= |k| <= kmax, amplitudes N(0, 1/8), phases U(0, 2 pi)."""
    rng = np.random.default_rng(seed)
    ks = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
          if 1 <= kx * kx + ky * ky <= kmax * kmax]
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    phi = np.zeros((n, n))
    for _ in range(modes):
        kx, ky = ks[rng.integers(len(ks))]
        a = rng.normal(0.0, np.sqrt(1.0 / 8.0))
        th = rng.uniform(0, 2 * np.pi)
        phi += a * np.cos(2 * np.pi * (kx * x + ky * y) / n + th)
    return 0.6 + 0.2 * np.tanh(phi)


def porosity_directions(n=256, count=16, first_seed=1):
    """Perturbation directions for gradient checks, each scaled to max |delta| = 1."""
    out = []
    for s in range(first_seed, first_seed + count):
        d = porosity_field(n, seed=s) - 0.6
        out.append(d / np.max(np.abs(d)))
    return out


def adjoint_cavity(n=256, storage="f32", seed=0):
    """Cavity with a spatially varying porosity field (Ra 1e5, Pr 1, Da 1e-2)."""
    cfg = cavity(n=n, eps=0.6, Da=1e-2, Ra=1e5, Pr=1.0, seed=seed, storage=storage)
    cfg["eps_field"] = porosity_field(n, seed=seed)
    return cfg


def ensemble(count=256, seed=0, side_lo=64, side_hi=512, storage="f32", max_cell_re=None):
    """Many cavities of uneven size and parameters: side N ~ U{lo..hi}, Da ~ 10^U(-4,-1),
    eps ~ U(0.4, 0.9), Pr = 1, and Ra log-uniform on [1e3, 1e6], or, with max_cell_re, on
    [1e3, min(1e6, Ra_max(N))] where Ra_max(N) = Pr (max_cell_re (N - 1))^2 keeps the grid
    cell Reynolds number sqrt(Ra / Pr) / (N - 1) at or below max_cell_re."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(side_lo, side_hi + 1))
        hi = 6.0 if max_cell_re is None else min(6.0, np.log10(1.0 * (max_cell_re * (n - 1)) ** 2))
        Ra = float(10 ** rng.uniform(3, max(3.0, hi)))
        Da = float(10 ** rng.uniform(-4, -1))
        eps = float(rng.uniform(0.4, 0.9))
        cfg = cavity(n=n, eps=eps, Da=Da, Ra=Ra, Pr=1.0, seed=seed * 100003 + k, storage=storage)
        out.append(cfg)
    return out


# ------------------------------------------------------------------------------------
# Three dimensions (D3Q19): periodic in x and y, walls at z = 0 and z = nz - 1 (or z
# periodic too).  Walls are listed bottom (z = 0) then top; "u" is the wall velocity.
# ------------------------------------------------------------------------------------
def layer3d(nx=64, ny=64, nz=32, eps=0.6, Da=1e-2, Ra=1e4, Pr=1.0, seed=0, storage="f64", amp=1e-3,
            tau=1.0, Ma=0.1):
    """Porous layer heated from below: isothermal walls, T_hot at z = 0 and T_cold at the
    top, buoyancy along +z, a conduction profile plus uniform noise of +-amp inside."""
    rng = np.random.default_rng(seed)
    z = np.arange(nz, dtype=np.float64) / (nz - 1)
    T = np.broadcast_to((1.0 - z)[:, None, None], (nz, ny, nx)).copy()
    T[1:-1] += rng.uniform(-amp, amp, size=(nz - 2, ny, nx))
    return {
        "nx": nx, "ny": ny, "nz": nz, "periodic_z": 0,
        "walls": [{"kind": "T", "T": 1.0}, {"kind": "T", "T": 0.0}],
        "Da": Da, "Ra": Ra, "Pr": Pr, "J": 1.0, "Ma": Ma, "sigma": 1.0, "Q": 0.0,
        "tau_f": tau, "tau_T": tau, "A": None, "B": None, "eps": eps, "a": (0.0, 0.0, 0.0),
        "T_hot": 1.0, "T_cold": 0.0, "F_eps": None, "T_init": T, "storage": storage,
    }


def random_case3d(seed, nx, ny, nz, periodic_z=0, storage="f64", eps_field=False, periodic_x=1, periodic_y=1):
    """A randomised 3-D problem with a non-trivial initial flow and temperature for parity
    tests: random Da, Ra in [1e2, 1e3], Pr, tau, A, B, eps, forcing and heat source, wall
    kinds and wall velocities, smooth random initial u and T; with eps_field, a smooth
    random porosity field in [0.4, 0.9]; with periodic_x = 0 (periodic_y = 0), walls at
    x = 0 and x = nx - 1 (y = 0 and y = ny - 1) of random kinds and tangential velocities
    (each drawn after everything before it, so a seed's earlier draws do not depend on these
    options)."""
    rng = np.random.default_rng(seed)
    tau_f, tau_T = rng.uniform(0.7, 1.3), rng.uniform(0.7, 1.3)
    walls = []
    for k in range(2):
        kind = "T" if rng.uniform() < 0.6 else "dTdn"
        walls.append({"kind": kind, "T": float(rng.uniform(0.0, 1.0)), "dTdn": float(rng.uniform(-0.01, 0.01)),
                      "u": tuple(float(v) for v in rng.uniform(-0.02, 0.02, size=3) * np.array([1.0, 1.0, 0.0]))})
    shape = (nz, ny, nx)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    def smooth(amp):
        f = np.zeros(shape)
        for _ in range(3):
            kx, ky, kz = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi, size=3)
            f += np.cos(2 * np.pi * kx * xx / nx + ph[0]) * np.cos(2 * np.pi * ky * yy / ny + ph[1]) \
                * np.cos(np.pi * kz * zz / max(nz - 1, 1) + ph[2])
        return amp * f / max(np.abs(f).max(), 1e-30)
    u = np.stack([smooth(0.02), smooth(0.02), smooth(0.01)])
    T = 0.5 + smooth(0.3)
    cfg = {
        "nx": nx, "ny": ny, "nz": nz, "periodic_z": periodic_z, "walls": walls,
        "L": 200.0, "Da": float(10 ** rng.uniform(-3, -1)), "Ra": float(10 ** rng.uniform(2, 3)),
        "Pr": float(rng.uniform(0.7, 2.0)), "J": 1.0, "Ma": 0.1, "sigma": float(rng.uniform(0.8, 1.2)),
        "Q": float(rng.uniform(0.0, 1e-5)), "tau_f": tau_f, "tau_T": tau_T,
        "A": float(rng.uniform(-0.1, tau_f - 0.55)), "B": float(rng.uniform(-0.1, tau_T - 0.55)),
        "eps": float(rng.uniform(0.4, 0.95)), "a": tuple(float(v) for v in rng.uniform(-1e-5, 1e-5, size=3)),
        "T_hot": 1.0, "T_cold": 0.0, "F_eps": None, "T_init": T, "u_init": u, "storage": storage,
    }
    if eps_field:
        cfg["eps_field"] = 0.65 + smooth(0.25)
    if not periodic_x:
        cfg["periodic_x"] = 0
        for k in range(2):
            kind = "T" if rng.uniform() < 0.6 else "dTdn"
            walls.append({"kind": kind, "T": float(rng.uniform(0.0, 1.0)), "dTdn": float(rng.uniform(-0.01, 0.01)),
                          "u": tuple(float(v) for v in rng.uniform(-0.02, 0.02, size=3) * np.array([0.0, 1.0, 1.0]))})
    if not periodic_y:
        cfg["periodic_y"] = 0
        while len(walls) < 4:
            walls.append({})
        for k in range(2):
            kind = "T" if rng.uniform() < 0.6 else "dTdn"
            walls.append({"kind": kind, "T": float(rng.uniform(0.0, 1.0)), "dTdn": float(rng.uniform(-0.01, 0.01)),
                          "u": tuple(float(v) for v in rng.uniform(-0.02, 0.02, size=3) * np.array([1.0, 0.0, 1.0]))})
    return cfg


def cavity3d(n=40, ny=2, eps=0.6, Da=1e-2, Ra=1e5, Pr=1.0, seed=0, storage="f64", tau=1.0, Ma=0.1):
    """The porous cavity of Sec. 4.2 on the 3-D lattice: hot wall x = 0, cold wall x = n - 1,
    adiabatic walls z = 0 and z = n - 1 (buoyancy along +z), periodic in y over ny nodes; the
    2-D cavity's initial temperature repeated along y, so the flow stays uniform in y."""
    T2 = cavity_T_init(n, n, seed)                  # [z][x]
    T = np.repeat(T2[:, None, :], ny, axis=1)       # [z][y][x]
    return {
        "nx": n, "ny": ny, "nz": n, "periodic_x": 0, "periodic_z": 0,
        "walls": [{"kind": "dTdn", "dTdn": 0.0}, {"kind": "dTdn", "dTdn": 0.0},
                  {"kind": "T", "T": 1.0}, {"kind": "T", "T": 0.0}],
        "Da": Da, "Ra": Ra, "Pr": Pr, "J": 1.0, "Ma": Ma, "sigma": 1.0, "Q": 0.0,
        "tau_f": tau, "tau_T": tau, "A": None, "B": None, "eps": eps, "a": (0.0, 0.0, 0.0),
        "T_hot": 1.0, "T_cold": 0.0, "F_eps": None, "T_init": T, "storage": storage,
    }
