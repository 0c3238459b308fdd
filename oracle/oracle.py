"""Python handle on the C oracle (TEST INFRASTRUCTURE ONLY).

The oracle is the plain FP64 CPU implementation of the modified lattice-BGK model for
convection heat transfer in porous media (Wang, Mi & Guo, arXiv:1505.02976) that the GPU
path is checked against.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import this module.  It never imports the GPU package and the GPU
package never imports it.

A problem is described by the same plain dictionary the GPU binding takes (see
``workloads.py``); this module turns it into the oracle's own C struct.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
LIB_REAL = os.path.join(_HERE, "liblbm_oracle.so")
LIB_COMPLEX = os.path.join(_HERE, "liblbm_oracle_cs.so")


def build(verbose: bool = False) -> None:
    """Compile both oracle variants (real and complex-step) with gcc."""
    base = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11", "-Wall",
            "-shared", "-fPIC"]
    for extra, out in (([], LIB_REAL), (["-DORC_COMPLEX"], LIB_COMPLEX)):
        cmd = base + extra + [_SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("wall_kind", C.c_int32 * 4),
        ("wall_ux", C.c_double * 4), ("wall_uy", C.c_double * 4),
        ("wall_T", C.c_double * 4), ("wall_dTdn", C.c_double * 4),
        ("L", C.c_double), ("Da", C.c_double), ("Ra", C.c_double), ("Pr", C.c_double),
        ("J", C.c_double), ("Ma", C.c_double), ("sigma", C.c_double), ("Q", C.c_double),
        ("tau_f", C.c_double), ("tau_T", C.c_double), ("A", C.c_double), ("B", C.c_double),
        ("eps", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
        ("T_hot", C.c_double), ("T_cold", C.c_double), ("F_eps", C.c_double),
    ]


def _params_from_dict(d: dict) -> _Params:
    p = _Params()
    p.nx, p.ny = int(d["nx"]), int(d["ny"])
    p.periodic_x, p.periodic_y = int(d.get("periodic_x", 0)), int(d.get("periodic_y", 0))
    walls = d.get("walls", [{}] * 4)
    for k in range(4):
        w = walls[k] if walls[k] is not None else {}
        p.wall_kind[k] = 1 if w.get("kind", "T") == "dTdn" else 0
        p.wall_ux[k] = float(w.get("ux", 0.0))
        p.wall_uy[k] = float(w.get("uy", 0.0))
        p.wall_T[k] = float(w.get("T", 0.0))
        p.wall_dTdn[k] = float(w.get("dTdn", 0.0))
    nan = float("nan")
    p.L = float(d.get("L", 0.0))
    p.Da = float(d.get("Da", math.inf))
    p.Ra = float(d.get("Ra", 0.0))
    p.Pr = float(d.get("Pr", 1.0))
    p.J = float(d.get("J", 1.0))
    p.Ma = float(d.get("Ma", 0.1))
    p.sigma = float(d.get("sigma", 1.0))
    p.Q = float(d.get("Q", 0.0))
    p.tau_f = float(d.get("tau_f", 1.0))
    p.tau_T = float(d.get("tau_T", 1.0))
    A = d.get("A", None)
    B = d.get("B", None)
    p.A = nan if A is None else float(A)
    p.B = nan if B is None else float(B)
    p.eps = float(d.get("eps", 1.0))
    p.ax = float(d.get("ax", 0.0))
    p.ay = float(d.get("ay", 0.0))
    p.T_hot = float(d.get("T_hot", 1.0))
    p.T_cold = float(d.get("T_cold", 0.0))
    Fe = d.get("F_eps", None)
    p.F_eps = nan if Fe is None else float(Fe)
    return p


_libs: dict = {}


def _lib(complex_step: bool):
    path = LIB_COMPLEX if complex_step else LIB_REAL
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [C.POINTER(_Params), vp, vp, vp, vp, vp]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_step.argtypes = [vp, C.c_int64]
    lib.orc_time.restype = C.c_int64
    lib.orc_time.argtypes = [vp]
    lib.orc_macro_fields.argtypes = [vp] + [vp] * 9
    lib.orc_get_populations.argtypes = [vp, C.c_int, vp, vp]
    lib.orc_set_post_populations.argtypes = [vp, vp, vp]
    lib.orc_nusselt.argtypes = [vp, C.c_int, vp]
    lib.orc_residual.restype = C.c_int
    lib.orc_residual.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.orc_lattice.argtypes = [vp, vp, vp]
    lib.orc_derive.restype = C.c_int
    lib.orc_derive.argtypes = [C.POINTER(_Params), vp]
    lib.orc_node_macro.argtypes = [C.POINTER(_Params), C.c_double, vp, vp, vp]
    lib.orc_node_terms.argtypes = [C.POINTER(_Params)] + [C.c_double] * 12 + [vp]
    lib.orc_node_collide.argtypes = [C.POINTER(_Params), C.c_double, vp, vp, vp, vp]
    _libs[path] = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lattice():
    """(cx, cy, w) as built by the oracle from the paper's D2Q9 definition."""
    lib = _lib(False)
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    w = np.zeros(9)
    lib.orc_lattice(_ptr(cx), _ptr(cy), _ptr(w))
    return cx, cy, w


DERIVED_KEYS = ("L", "A", "B", "nu_e", "nu", "alpha_e", "gbeta", "K", "T0", "dT")


def derived(cfg: dict) -> dict:
    """Lattice constants the oracle derives from a problem description."""
    lib = _lib(False)
    out = np.zeros(10)
    p = _params_from_dict(cfg)
    rc = lib.orc_derive(C.byref(p), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle rejected parameters (code {rc})")
    return dict(zip(DERIVED_KEYS, out.tolist()))


class Oracle:
    """One simulation held by the C oracle.

    Fields are numpy arrays shaped [ny, nx]; with ``complex_step=True`` every array is
    complex128 and the porosity field may carry an imaginary perturbation.
    """

    def __init__(self, cfg: dict, complex_step: bool = False):
        self.cfg = cfg
        self.cs = complex_step
        self.dtype = np.complex128 if complex_step else np.float64
        self.lib = _lib(complex_step)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self._p = _params_from_dict(cfg)

        def arr(key):
            a = cfg.get(key, None)
            if a is None:
                return None
            a = np.ascontiguousarray(np.asarray(a, dtype=self.dtype).reshape(self.ny, self.nx))
            return a

        self._keep = [arr(k) for k in ("eps_field", "T_init", "p_init", "ux_init", "uy_init")]
        h = self.lib.orc_create(C.byref(self._p), *[_ptr(a) for a in self._keep])
        if not h:
            raise ValueError("oracle rejected parameters")
        self.h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    @property
    def time(self) -> int:
        return int(self.lib.orc_time(self.h))

    def step(self, n: int = 1) -> None:
        self.lib.orc_step(self.h, int(n))

    def fields(self) -> dict:
        names = ("p", "ux", "uy", "T", "Sxx", "Sxy", "Syy", "dTdx", "dTdy")
        out = {k: np.zeros((self.ny, self.nx), self.dtype) for k in names}
        self.lib.orc_macro_fields(self.h, *[_ptr(out[k]) for k in names])
        return out

    def populations(self, post: bool = True):
        """(f, g), each [9, ny, nx]: post-collision of the last step, or pre-collision now."""
        f = np.zeros((9, self.ny, self.nx), self.dtype)
        g = np.zeros((9, self.ny, self.nx), self.dtype)
        self.lib.orc_get_populations(self.h, 1 if post else 0, _ptr(f), _ptr(g))
        return f, g

    def set_post_populations(self, f, g) -> None:
        f = np.ascontiguousarray(f, dtype=self.dtype)
        g = np.ascontiguousarray(g, dtype=self.dtype)
        self.lib.orc_set_post_populations(self.h, _ptr(f), _ptr(g))

    def nusselt(self, wall: int = 0):
        out = np.zeros(1, self.dtype)
        self.lib.orc_nusselt(self.h, int(wall), _ptr(out))
        return out[0]

    def residual(self):
        ru, rT = C.c_double(), C.c_double()
        rc = self.lib.orc_residual(self.h, C.byref(ru), C.byref(rT))
        return (None, None) if rc == 1 else (ru.value, rT.value)

    def run_to_steady(self, tol: float, max_steps: int, every: int = 100):
        """Step until both residuals (against the state `every` steps earlier) fall below tol."""
        self.residual()
        while self.time < max_steps:
            self.step(every)
            ru, rT = self.residual()
            if ru < tol and rT < tol:
                return True
        return False


def node_macro(cfg: dict, eps: float, f, g):
    """Macroscopic quantities at one node: dict of T, G, v, u, F, p, S, grad T."""
    lib = _lib(False)
    p = _params_from_dict(cfg)
    f = np.ascontiguousarray(f, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    out = np.zeros(16)
    lib.orc_node_macro(C.byref(p), float(eps), _ptr(f), _ptr(g), _ptr(out))
    keys = ("T", "Gx", "Gy", "vx", "vy", "ux", "uy", "Fx", "Fy", "p",
            "Sxx", "Sxy", "Syy", "dTdx", "dTdy", "eps")
    return dict(zip(keys, out.tolist()))


def node_terms(cfg: dict, eps, T, ux, uy, p, Sxx, Sxy, Syy, dTx, dTy, Fx, Fy):
    """Discrete terms at one node: dict of arrays feq0, r, geq0, gB, F, P, Q (each 9)."""
    lib = _lib(False)
    prm = _params_from_dict(cfg)
    out = np.zeros(63)
    lib.orc_node_terms(C.byref(prm), *[float(v) for v in
                                       (eps, T, ux, uy, p, Sxx, Sxy, Syy, dTx, dTy, Fx, Fy)],
                       _ptr(out))
    names = ("feq0", "r", "geq0", "gB", "F", "P", "Q")
    return {k: out[9 * i:9 * i + 9].copy() for i, k in enumerate(names)}


def node_collide(cfg: dict, eps: float, f, g):
    lib = _lib(False)
    prm = _params_from_dict(cfg)
    f = np.ascontiguousarray(f, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    fo = np.zeros(9)
    go = np.zeros(9)
    lib.orc_node_collide(C.byref(prm), float(eps), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    return fo, go
