"""Python handle on the 3-D C oracle (TEST INFRASTRUCTURE ONLY).

The plain FP64 CPU implementation of the modified lattice-BGK model on the D3Q19 lattice
(x, y and z each periodic or walled) that the GPU path's 3-D kernels are
checked against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; it never imports the GPU package.

A problem is the plain dictionary of ``workloads.layer3d`` / ``workloads.random_case3d``
(the GPU binding takes the same).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm3_oracle.c")
LIB = os.path.join(_HERE, "liblbm3_oracle.so")
_lib_handle = None


def build(verbose: bool = False) -> None:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11", "-Wall", "-shared", "-fPIC",
           _SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("periodic_x", C.c_int32),
        ("periodic_y", C.c_int32), ("periodic_z", C.c_int32),
        ("wall_kind", C.c_int32 * 6),
        ("wall_u", (C.c_double * 3) * 6),
        ("wall_T", C.c_double * 6), ("wall_dTdn", C.c_double * 6),
        ("L", C.c_double), ("Da", C.c_double), ("Ra", C.c_double), ("Pr", C.c_double),
        ("J", C.c_double), ("Ma", C.c_double), ("sigma", C.c_double), ("Q", C.c_double),
        ("tau_f", C.c_double), ("tau_T", C.c_double), ("A", C.c_double), ("B", C.c_double),
        ("eps", C.c_double), ("a", C.c_double * 3),
        ("T_hot", C.c_double), ("T_cold", C.c_double), ("F_eps", C.c_double),
    ]


def _nan(v):
    return math.nan if v is None else float(v)


def params_from_dict(d: dict) -> _Params:
    p = _Params()
    p.nx, p.ny, p.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
    p.periodic_z = int(d.get("periodic_z", 0))
    p.periodic_x = int(d.get("periodic_x", 1))
    p.periodic_y = int(d.get("periodic_y", 1))
    for k, w in enumerate(d["walls"]):
        p.wall_kind[k] = 1 if w.get("kind", "T") == "dTdn" else 0
        for a, v in enumerate(w.get("u", (0.0, 0.0, 0.0))):
            p.wall_u[k][a] = float(v)
        p.wall_T[k] = float(w.get("T", 0.0))
        p.wall_dTdn[k] = float(w.get("dTdn", 0.0))
    p.L = float(d.get("L", 0.0) or 0.0)
    for key in ("Da", "Ra", "Pr", "J", "Ma", "sigma", "Q", "tau_f", "tau_T", "eps", "T_hot", "T_cold"):
        setattr(p, key, float(d[key]))
    p.A, p.B, p.F_eps = _nan(d.get("A")), _nan(d.get("B")), _nan(d.get("F_eps"))
    for a, v in enumerate(d.get("a", (0.0, 0.0, 0.0))):
        p.a[a] = float(v)
    return p


def _lib():
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(_SRC):
        build()
    L = C.CDLL(LIB)
    vp = C.c_void_p
    L.o3_create.restype = vp
    L.o3_create.argtypes = [C.POINTER(_Params), vp, vp, vp]
    L.o3_destroy.argtypes = [vp]
    L.o3_step.argtypes = [vp, C.c_int64]
    L.o3_fields.argtypes = [vp] * 6
    L.o3_get_populations.argtypes = [vp, C.c_int, vp, vp]
    L.o3_nusselt.restype = C.c_double
    L.o3_nusselt.argtypes = [vp, C.c_int]
    L.o3_lattice.argtypes = [vp, vp]
    L.o3_derive.restype = C.c_int
    L.o3_derive.argtypes = [C.POINTER(_Params), vp]
    L.o3_node_macro.restype = C.c_int
    L.o3_node_macro.argtypes = [C.POINTER(_Params), C.c_double, vp, vp, vp]
    L.o3_node_terms.restype = C.c_int
    L.o3_node_terms.argtypes = [C.POINTER(_Params), C.c_double, C.c_double, vp, C.c_double, vp, vp, vp, vp]
    L.o3_node_collide.restype = C.c_int
    L.o3_node_collide.argtypes = [C.POINTER(_Params), C.c_double, vp, vp, vp, vp]
    _lib_handle = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lattice():
    """(c [19, 3] int, w [19]) of the oracle's D3Q19 lattice."""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    _lib().o3_lattice(_ptr(c), _ptr(w))
    return c, w


def derived(cfg: dict) -> dict:
    out = np.zeros(10)
    r = _lib().o3_derive(C.byref(params_from_dict(cfg)), _ptr(out))
    if r != 0:
        raise ValueError(f"oracle rejected parameters ({r})")
    return dict(zip(("L", "A", "B", "nu_e", "nu", "alpha_e", "gbeta", "K", "T0", "dT"), out.tolist()))


class Oracle3:
    """One 3-D simulation; fields are numpy arrays shaped [nz, ny, nx]."""

    def __init__(self, cfg: dict):
        self.cfg = cfg
        self.lib = _lib()
        self.shape = (int(cfg["nz"]), int(cfg["ny"]), int(cfg["nx"]))
        self.n = int(np.prod(self.shape))
        self._p = params_from_dict(cfg)
        e = cfg.get("eps_field")
        T = cfg.get("T_init")
        u = cfg.get("u_init")
        self._keep = [None if e is None else np.ascontiguousarray(np.asarray(e, np.float64).reshape(self.shape)),
                      None if T is None else np.ascontiguousarray(np.asarray(T, np.float64).reshape(self.shape)),
                      None if u is None else np.ascontiguousarray(np.asarray(u, np.float64).reshape((3,) + self.shape))]
        h = self.lib.o3_create(C.byref(self._p), *[_ptr(a) for a in self._keep])
        if not h:
            raise ValueError("oracle rejected parameters")
        self.h = C.c_void_p(h)
        self.time = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.o3_destroy(h)
            self.h = None

    def step(self, n: int = 1) -> None:
        self.lib.o3_step(self.h, int(n))
        self.time += int(n)

    def fields(self) -> dict:
        p = np.zeros(self.shape)
        T = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        S = np.zeros((6,) + self.shape)
        dT = np.zeros((3,) + self.shape)
        self.lib.o3_fields(self.h, _ptr(p), _ptr(u), _ptr(T), _ptr(S), _ptr(dT))
        out = {"p": p, "T": T}
        out.update({k: u[a] for a, k in enumerate(("ux", "uy", "uz"))})
        out.update({k: S[c] for c, k in enumerate(("Sxx", "Sxy", "Sxz", "Syy", "Syz", "Szz"))})
        out.update({k: dT[a] for a, k in enumerate(("dTdx", "dTdy", "dTdz"))})
        return out

    def populations(self, post: bool = False):
        """(f, g), each [19, nz, ny, nx] in the oracle's lattice order."""
        f = np.zeros((19,) + self.shape)
        g = np.zeros((19,) + self.shape)
        self.lib.o3_get_populations(self.h, 1 if post else 0, _ptr(f), _ptr(g))
        return f, g

    def nusselt(self, wall: int = 0) -> float:
        return float(self.lib.o3_nusselt(self.h, int(wall)))


def _vec(v, n):
    a = np.ascontiguousarray(np.asarray(v, np.float64).reshape(n))
    return a


def node_macro(cfg: dict, eps: float, f, g) -> dict:
    """Macroscopic state of one bulk node from its pre-collision populations f[19], g[19]:
    T, G (3), u (3), F (3), p, S (3 x 3), grad T (3)."""
    f, g = _vec(f, 19), _vec(g, 19)
    out = np.zeros(23)
    _lib().o3_node_macro(C.byref(params_from_dict(cfg)), float(eps), _ptr(f), _ptr(g), _ptr(out))
    return {"T": out[0], "G": out[1:4].copy(), "u": out[4:7].copy(), "F": out[7:10].copy(),
            "p": out[10], "S": out[11:20].reshape(3, 3).copy(), "dT": out[20:23].copy()}


def node_terms(cfg: dict, eps, T, u, p, S, dT, F) -> dict:
    """Discrete terms of one node for prescribed macroscopic values: arrays of 19 for
    feq0, r, geq0, gB, F, P, Q."""
    u, S, dT, F = _vec(u, 3), _vec(S, 9), _vec(dT, 3), _vec(F, 3)
    out = np.zeros(7 * 19)
    _lib().o3_node_terms(C.byref(params_from_dict(cfg)), float(eps), float(T), _ptr(u), float(p), _ptr(S),
                         _ptr(dT), _ptr(F), _ptr(out))
    names = ("feq0", "r", "geq0", "gB", "F", "P", "Q")
    return {k: out[19 * i:19 * i + 19].copy() for i, k in enumerate(names)}


def node_collide(cfg: dict, eps: float, f, g):
    """Post-collision populations (fo, go) of one bulk node."""
    f, g = _vec(f, 19), _vec(g, 19)
    fo, go = np.zeros(19), np.zeros(19)
    _lib().o3_node_collide(C.byref(params_from_dict(cfg)), float(eps), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    return fo, go
