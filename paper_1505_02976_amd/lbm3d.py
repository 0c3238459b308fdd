"""ctypes binding of the three-dimensional entry points (include/lbm3d.h): argument
marshalling only; every step runs in the library's kernels.  A problem is the plain
dictionary of ``workloads.layer3d`` / ``workloads.random_case3d`` / ``workloads.cavity3d``; fields come back as
torch tensors shaped [nz, ny, nx] (vector and tensor fields as stacked planes)."""
from __future__ import annotations

import ctypes as C
import math

from . import lbm as _lbm

STORAGE3 = {"f64": 0, "f32": 1, "f16": 2}


class _Wall3(C.Structure):
    _fields_ = [("u", C.c_double * 3), ("t_kind", C.c_int32), ("reserved", C.c_int32),
                ("T", C.c_double), ("dTdn", C.c_double)]


class _Params3(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("periodic_x", C.c_int32),
        ("periodic_y", C.c_int32), ("periodic_z", C.c_int32),
        ("wall", _Wall3 * 6),
        ("L", C.c_double), ("Da", C.c_double), ("Ra", C.c_double), ("Pr", C.c_double),
        ("J", C.c_double), ("Ma", C.c_double), ("sigma", C.c_double), ("Q", C.c_double),
        ("tau_f", C.c_double), ("tau_T", C.c_double), ("A", C.c_double), ("B", C.c_double),
        ("eps", C.c_double), ("a", C.c_double * 3),
        ("T_hot", C.c_double), ("T_cold", C.c_double), ("F_eps", C.c_double),
        ("storage", C.c_int32), ("reserved", C.c_int32),
        ("T_init", C.c_void_p), ("u_init", C.c_void_p), ("eps_field", C.c_void_p),
    ]


_ready = False


def lib():
    """The library with the 3-D entry points typed."""
    global _ready
    L = _lbm.lib()
    if not _ready:
        vp = C.c_void_p
        L.lbm3_workspace_bytes.restype = C.c_size_t
        L.lbm3_workspace_bytes.argtypes = [C.POINTER(_Params3)]
        L.lbm3_init.restype = C.c_int
        L.lbm3_init.argtypes = [C.POINTER(_Params3), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm3_step.restype = C.c_int
        L.lbm3_step.argtypes = [vp, C.c_int64]
        L.lbm3_fields.restype = C.c_int
        L.lbm3_fields.argtypes = [vp] * 6
        L.lbm3_populations.restype = C.c_int
        L.lbm3_populations.argtypes = [vp, vp, vp]
        L.lbm3_nusselt.restype = C.c_int
        L.lbm3_nusselt.argtypes = [vp, C.c_int32, C.POINTER(C.c_double)]
        L.lbm3_lattice.restype = C.c_int32
        L.lbm3_lattice.argtypes = [vp]
        L.lbm3_time.restype = C.c_int64
        L.lbm3_time.argtypes = [vp]
        L.lbm3_destroy.argtypes = [vp]
        _ready = True
    return L


def _f(v):
    return math.nan if v is None else float(v)


def make_params(cfg: dict, T_init=0, u_init=0, eps_field=0) -> _Params3:
    p = _Params3()
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
    p.periodic_x = int(cfg.get("periodic_x", 1))
    p.periodic_y = int(cfg.get("periodic_y", 1))
    p.periodic_z = int(cfg.get("periodic_z", 0))
    for k, w in enumerate(cfg["walls"]):
        p.wall[k].t_kind = 1 if w.get("kind", "T") == "dTdn" else 0
        for a, v in enumerate(w.get("u", (0.0, 0.0, 0.0))):
            p.wall[k].u[a] = float(v)
        p.wall[k].T = float(w.get("T", 0.0))
        p.wall[k].dTdn = float(w.get("dTdn", 0.0))
    p.L = float(cfg.get("L", 0.0) or 0.0)
    for key in ("Da", "Ra", "Pr", "J", "Ma", "sigma", "Q", "tau_f", "tau_T", "eps", "T_hot", "T_cold"):
        setattr(p, key, float(cfg[key]))
    p.A, p.B, p.F_eps = _f(cfg.get("A")), _f(cfg.get("B")), _f(cfg.get("F_eps"))
    for a, v in enumerate(cfg.get("a", (0.0, 0.0, 0.0))):
        p.a[a] = float(v)
    p.storage = STORAGE3[cfg.get("storage", "f64")]
    p.T_init = T_init or None
    p.u_init = u_init or None
    p.eps_field = eps_field or None
    return p


def lattice():
    """The library's D3Q19 velocities in population order, as a list of 19 (cx, cy, cz)."""
    c = (C.c_int32 * 57)()
    lib().lbm3_lattice(c)
    return [tuple(c[3 * i:3 * i + 3]) for i in range(19)]


def workspace_bytes(cfg: dict) -> int:
    return int(lib().lbm3_workspace_bytes(C.byref(make_params(cfg))))


class Sim3:
    """One 3-D problem on one GPU (workspace from torch, launches on torch's current stream)."""

    def __init__(self, cfg: dict, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.shape = (int(cfg["nz"]), int(cfg["ny"]), int(cfg["nx"]))
        L = lib()
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            keep = []
            ptrs = {}
            for key, shp in (("T_init", self.shape), ("u_init", (3,) + self.shape)):
                a = cfg.get(key)
                if a is not None:
                    t = torch.as_tensor(a, dtype=torch.float64).reshape(shp).contiguous().to(self.device)
                    keep.append(t)
                    ptrs[key] = t.data_ptr()
            # the porosity field is read by every step: it lives as long as the simulation
            self.eps_field = None
            if cfg.get("eps_field") is not None:
                self.eps_field = torch.as_tensor(cfg["eps_field"], dtype=torch.float64).reshape(
                    self.shape).contiguous().to(self.device)
            p = make_params(cfg, ptrs.get("T_init", 0), ptrs.get("u_init", 0),
                            self.eps_field.data_ptr() if self.eps_field is not None else 0)
            nbytes = int(L.lbm3_workspace_bytes(C.byref(p)))
            if nbytes == 0:
                raise _lbm.LbmError(_lbm.ERR_INVALID, L.lbm_last_error().decode())
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.workspace.data_ptr() + 255) // 256 * 256
            h = C.c_void_p()
            _lbm._check(L.lbm3_init(C.byref(p), C.c_void_p(aligned), nbytes, C.c_void_p(self.stream.cuda_stream),
                                    C.byref(h)))
            self.h = h
            del keep

    @property
    def time(self) -> int:
        return int(lib().lbm3_time(self.h))

    def step(self, n: int = 1) -> None:
        _lbm._check(lib().lbm3_step(self.h, int(n)))

    def fields(self) -> dict:
        t = self.torch
        o = {"p": t.empty(self.shape, dtype=t.float64, device=self.device),
             "T": t.empty(self.shape, dtype=t.float64, device=self.device),
             "u": t.empty((3,) + self.shape, dtype=t.float64, device=self.device),
             "S": t.empty((6,) + self.shape, dtype=t.float64, device=self.device),
             "gT": t.empty((3,) + self.shape, dtype=t.float64, device=self.device)}
        _lbm._check(lib().lbm3_fields(self.h, *[o[k].data_ptr() for k in ("p", "u", "T", "S", "gT")]))
        self.stream.synchronize()
        out = {"p": o["p"], "T": o["T"]}
        out.update({k: o["u"][a] for a, k in enumerate(("ux", "uy", "uz"))})
        out.update({k: o["S"][c] for c, k in enumerate(("Sxx", "Sxy", "Sxz", "Syy", "Syz", "Szz"))})
        out.update({k: o["gT"][a] for a, k in enumerate(("dTdx", "dTdy", "dTdz"))})
        return out

    def nusselt(self, wall: int = 0) -> float:
        """Average Nusselt number of wall 0 (z = 0), 1 (z = nz - 1), 2 (x = 0), 3 (x = nx - 1),
        4 (y = 0) or 5 (y = ny - 1), FP64."""
        v = C.c_double()
        _lbm._check(lib().lbm3_nusselt(self.h, int(wall), C.byref(v)))
        return v.value

    def populations(self):
        """(f, g) pre-collision now, each [19, nz, ny, nx] in the order of lattice()."""
        t = self.torch
        f = t.empty((19,) + self.shape, dtype=t.float64, device=self.device)
        g = t.empty((19,) + self.shape, dtype=t.float64, device=self.device)
        _lbm._check(lib().lbm3_populations(self.h, f.data_ptr(), g.data_ptr()))
        self.stream.synchronize()
        return f, g

    def close(self):
        h = getattr(self, "h", None)
        if h:
            lib().lbm3_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:      # interpreter shutdown: the module's globals may be gone
            pass
