"""Python binding of the C interface in include/lbm.h (argument marshalling only).

PyTorch supplies device memory (the workspace and field buffers) and the HIP stream;
every step of the method runs in the HIP kernels of liblbm.so.  The binding refuses to
run when the library is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

OK, ERR_INVALID, ERR_DEVICE, ERR_NONFINITE, ERR_UNSUPPORTED = 0, 1, 2, 3, 4
STORAGE = {"f64": 0, "f32": 1, "f16": 2}


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


class NonFiniteError(LbmError):
    pass


class _Wall(C.Structure):
    _fields_ = [("ux", C.c_double), ("uy", C.c_double), ("t_kind", C.c_int32),
                ("reserved", C.c_int32), ("T", C.c_double), ("dTdn", C.c_double)]


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("wall", _Wall * 4),
        ("L", C.c_double), ("Da", C.c_double), ("Ra", C.c_double), ("Pr", C.c_double),
        ("J", C.c_double), ("Ma", C.c_double), ("sigma", C.c_double), ("Q", C.c_double),
        ("tau_f", C.c_double), ("tau_T", C.c_double), ("A", C.c_double), ("B", C.c_double),
        ("eps", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
        ("T_hot", C.c_double), ("T_cold", C.c_double), ("F_eps", C.c_double),
        ("eps_field", C.c_void_p), ("T_init", C.c_void_p), ("p_init", C.c_void_p),
        ("ux_init", C.c_void_p), ("uy_init", C.c_void_p),
        ("storage", C.c_int32), ("reserved", C.c_int32),
    ]


class _Derived(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("L", "A", "B", "nu_e", "nu", "alpha_e", "gbeta", "K", "T0", "dT")]


_lib = None

EXPORTS = ("lbm_derive", "lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_step_timed", "lbm_time",
           "lbm_moments", "lbm_gradients", "lbm_nusselt", "lbm_residual", "lbm_get_state",
           "lbm_set_state", "lbm_destroy", "lbm_last_error", "lbm_set_fusion", "lbm_fusion",
           "lbm_batch_workspace_bytes", "lbm_batch_init", "lbm_batch_step", "lbm_batch_problem",
           "lbm_batch_check", "lbm_batch_destroy", "lbm_batch_autotune",
           "lbm_batch_set_width", "lbm_batch_set_fusion", "lbm_batch_fusion",
           "lbm_adjoint_workspace_bytes", "lbm_adjoint_forward", "lbm_adjoint_backward",
           "lbm_adjoint_destroy", "lbm_residual_noalloc", "lbm_set_check_interval")


def lib():
    """Loads liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1505_02976_amd.build.build()")
    # torch first: it loads its own HIP and HSA runtimes (same sonames as the system's), and the
    # library must bind to those.  Loaded the other way round the process holds two of each,
    # and device memory from torch is not valid in the library's runtime.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_derive.restype = st
    L.lbm_derive.argtypes = [C.POINTER(_Params), C.POINTER(_Derived)]
    L.lbm_workspace_bytes.restype = C.c_size_t
    L.lbm_workspace_bytes.argtypes = [C.POINTER(_Params)]
    L.lbm_init.restype = st
    L.lbm_init.argtypes = [C.POINTER(_Params), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lbm_step.restype = st
    L.lbm_step.argtypes = [vp, C.c_int64]
    L.lbm_step_timed.restype = st
    L.lbm_step_timed.argtypes = [vp, C.c_int64, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    L.lbm_set_fusion.restype = st
    L.lbm_set_fusion.argtypes = [vp, C.c_int32]
    L.lbm_fusion.restype = C.c_int32
    L.lbm_fusion.argtypes = [vp]
    L.lbm_time.restype = C.c_int64
    L.lbm_time.argtypes = [vp]
    L.lbm_moments.restype = st
    L.lbm_moments.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.lbm_gradients.restype = st
    L.lbm_gradients.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp]
    L.lbm_nusselt.restype = st
    L.lbm_nusselt.argtypes = [vp, C.c_int32, C.POINTER(C.c_double)]
    L.lbm_residual.restype = st
    L.lbm_residual.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.lbm_set_check_interval.restype = st
    L.lbm_set_check_interval.argtypes = [vp, C.c_int64]
    L.lbm_residual_noalloc.restype = st
    L.lbm_residual_noalloc.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.lbm_get_state.restype = st
    L.lbm_get_state.argtypes = [vp, vp]
    L.lbm_set_state.restype = st
    L.lbm_set_state.argtypes = [vp, vp]
    L.lbm_destroy.restype = None
    L.lbm_destroy.argtypes = [vp]
    L.lbm_batch_workspace_bytes.restype = C.c_size_t
    L.lbm_batch_workspace_bytes.argtypes = [C.POINTER(_Params), C.c_int32]
    L.lbm_batch_init.restype = st
    L.lbm_batch_init.argtypes = [C.POINTER(_Params), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lbm_batch_step.restype = st
    L.lbm_batch_step.argtypes = [vp, C.c_int64]
    L.lbm_batch_problem.restype = vp
    L.lbm_batch_problem.argtypes = [vp, C.c_int32]
    L.lbm_batch_check.restype = st
    L.lbm_batch_check.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lbm_batch_autotune.restype = st
    L.lbm_batch_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.lbm_batch_set_width.restype = st
    L.lbm_batch_set_width.argtypes = [vp, C.c_int32]
    L.lbm_batch_set_fusion.restype = st
    L.lbm_batch_set_fusion.argtypes = [vp, C.c_int32]
    L.lbm_batch_fusion.restype = C.c_int32
    L.lbm_batch_fusion.argtypes = [vp]
    L.lbm_batch_destroy.restype = None
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_adjoint_workspace_bytes.restype = C.c_size_t
    L.lbm_adjoint_workspace_bytes.argtypes = [vp, C.c_int64]
    L.lbm_adjoint_forward.restype = st
    L.lbm_adjoint_forward.argtypes = [vp, C.c_int32, C.c_int64, vp, C.c_size_t, C.POINTER(vp),
                                      C.POINTER(C.c_double)]
    L.lbm_adjoint_backward.restype = st
    L.lbm_adjoint_backward.argtypes = [vp, C.c_double, vp]
    L.lbm_adjoint_destroy.restype = None
    L.lbm_adjoint_destroy.argtypes = [vp]
    _lib = L
    return L


def _check(status):
    if status != OK:
        msg = lib().lbm_last_error().decode()
        if status == ERR_NONFINITE:
            raise NonFiniteError(status, msg)
        raise LbmError(status, msg)


def make_params(cfg: dict, fields: dict | None = None) -> _Params:
    """Fills the C parameter block from a problem dictionary (see workloads.py);
    `fields` maps eps_field/T_init/p_init/ux_init/uy_init to device pointers."""
    p = _Params()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.periodic_x = int(cfg.get("periodic_x", 0))
    p.periodic_y = int(cfg.get("periodic_y", 0))
    walls = cfg.get("walls", [{}] * 4)
    for k in range(4):
        w = walls[k] or {}
        p.wall[k].ux = float(w.get("ux", 0.0))
        p.wall[k].uy = float(w.get("uy", 0.0))
        p.wall[k].t_kind = 1 if w.get("kind", "T") == "dTdn" else 0
        p.wall[k].T = float(w.get("T", 0.0))
        p.wall[k].dTdn = float(w.get("dTdn", 0.0))
    nan = float("nan")
    p.L = float(cfg.get("L", 0.0))
    p.Da = float(cfg.get("Da", math.inf))
    p.Ra = float(cfg.get("Ra", 0.0))
    p.Pr = float(cfg.get("Pr", 1.0))
    p.J = float(cfg.get("J", 1.0))
    p.Ma = float(cfg.get("Ma", 0.1))
    p.sigma = float(cfg.get("sigma", 1.0))
    p.Q = float(cfg.get("Q", 0.0))
    p.tau_f = float(cfg.get("tau_f", 1.0))
    p.tau_T = float(cfg.get("tau_T", 1.0))
    p.A = nan if cfg.get("A") is None else float(cfg["A"])
    p.B = nan if cfg.get("B") is None else float(cfg["B"])
    p.eps = float(cfg.get("eps", 1.0))
    p.ax = float(cfg.get("ax", 0.0))
    p.ay = float(cfg.get("ay", 0.0))
    p.T_hot = float(cfg.get("T_hot", 1.0))
    p.T_cold = float(cfg.get("T_cold", 0.0))
    p.F_eps = nan if cfg.get("F_eps") is None else float(cfg["F_eps"])
    p.storage = STORAGE[cfg.get("storage", "f64")]
    fields = fields or {}
    for key in ("eps_field", "T_init", "p_init", "ux_init", "uy_init"):
        setattr(p, key, fields.get(key))
    return p


def derived(cfg: dict) -> dict:
    d = _Derived()
    _check(lib().lbm_derive(C.byref(make_params(cfg)), C.byref(d)))
    return {k: getattr(d, k) for k, _ in _Derived._fields_}


def workspace_bytes(cfg: dict) -> int:
    return int(lib().lbm_workspace_bytes(C.byref(make_params(cfg))))


def _device_fields(torch, cfg, device, nx, ny):
    """Initial fields of a problem as FP64 device tensors (numpy arrays or torch tensors in
    the problem dictionary); returns (pointer map, tensors to keep alive)."""
    dev, keep = {}, []
    for key in ("eps_field", "T_init", "p_init", "ux_init", "uy_init"):
        a = cfg.get(key)
        if a is None:
            continue
        if isinstance(a, torch.Tensor):
            t = a.detach().to(device=device, dtype=torch.float64).reshape(ny, nx).contiguous()
        else:
            t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(ny, nx), device=device)
        keep.append(t)
        dev[key] = t.data_ptr()
    return dev, keep


class Sim:
    """A simulation context on a CUDA (HIP) device; fields come back as torch tensors."""

    @classmethod
    def _wrap(cls, handle, cfg, device, stream, owner):
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self.stream = stream
        self.h = C.c_void_p(handle)
        self._owner = owner      # the batch owns the context
        return self

    def __init__(self, cfg: dict, device: str = "cuda:0", stream=None):
        import torch
        self._owner = None
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        L = lib()
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            dev, keep = _device_fields(torch, cfg, self.device, self.nx, self.ny)
            prm = make_params(cfg, dev)
            nbytes = int(L.lbm_workspace_bytes(C.byref(prm)))
            if nbytes == 0:
                _check(L.lbm_derive(C.byref(prm), C.byref(_Derived())))
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
            h = C.c_void_p()
            _check(L.lbm_init(C.byref(prm), C.c_void_p(aligned), nbytes,
                              C.c_void_p(self.stream.cuda_stream), C.byref(h)))
            self.h = h
            # initial fields are read by the init kernel: wait before releasing them
            self.stream.synchronize()
            del keep

    def close(self):
        if getattr(self, "h", None) and getattr(self, "_owner", None) is None:
            lib().lbm_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self) -> int:
        return int(lib().lbm_time(self.h))

    def step(self, n: int = 1):
        _check(lib().lbm_step(self.h, int(n)))

    def step_timed(self, n: int, every: int = 1):
        """Steps with HIP events around the launches of every `every`-th pass; returns
        (main_ms, rest_ms, main_nodes, steps_per_pass): mean launch durations over the
        bracketed passes, the nodes the main launch updates and the steps one pass makes."""
        b, w, nodes, k = C.c_double(), C.c_double(), C.c_int64(), C.c_int32()
        _check(lib().lbm_step_timed(self.h, int(n), int(every), C.byref(b), C.byref(w), C.byref(nodes),
                                    C.byref(k)))
        return b.value, w.value, nodes.value, k.value

    @property
    def fusion(self) -> int:
        """Time steps per pass over the populations (1 or 2)."""
        return int(lib().lbm_fusion(self.h))

    @fusion.setter
    def fusion(self, steps_per_pass: int):
        _check(lib().lbm_set_fusion(self.h, int(steps_per_pass)))

    def _alloc(self, dtype):
        return self.torch.empty((self.ny, self.nx), dtype=dtype, device=self.device)

    def fields(self, f32: bool = False, gradients: bool = True) -> dict:
        dt = self.torch.float32 if f32 else self.torch.float64
        out = {k: self._alloc(dt) for k in ("p", "ux", "uy", "T")}
        _check(lib().lbm_moments(self.h, 1 if f32 else 0, *[out[k].data_ptr() for k in ("p", "ux", "uy", "T")]))
        if gradients:
            for k in ("Sxx", "Sxy", "Syy", "dTdx", "dTdy"):
                out[k] = self._alloc(dt)
            _check(lib().lbm_gradients(self.h, 1 if f32 else 0,
                                       *[out[k].data_ptr() for k in ("Sxx", "Sxy", "Syy", "dTdx", "dTdy")]))
        self.stream.synchronize()
        return out

    def nusselt(self, wall: int = 0) -> float:
        v = C.c_double()
        _check(lib().lbm_nusselt(self.h, int(wall), C.byref(v)))
        return v.value

    def residual(self):
        ru, rT = C.c_double(), C.c_double()
        _check(lib().lbm_residual(self.h, C.byref(ru), C.byref(rT)))
        return (None, None) if ru.value < 0 else (ru.value, rT.value)

    def set_check_interval(self, every: int):
        """Make step() wait and check for non-finite populations whenever the time reaches a
        multiple of `every` (0: never); a failing check raises LbmError (LBM_ERR_NONFINITE)."""
        _check(lib().lbm_set_check_interval(self.h, int(every)))

    def residual_noalloc(self):
        """As residual, with the reduction's scratch in the library's static device array
        (lbm_residual_noalloc): allocates nothing."""
        ru, rT = C.c_double(), C.c_double()
        _check(lib().lbm_residual_noalloc(self.h, C.byref(ru), C.byref(rT)))
        return (None, None) if ru.value < 0 else (ru.value, rT.value)

    def run_to_steady(self, tol: float, max_steps: int, every: int = 100) -> bool:
        """Steps until both residuals of Sec. 4 (against the state `every` steps earlier) fall
        below tol or the time reaches max_steps; returns whether they did.  The last pair of
        residuals is kept in self.last_residual."""
        self.residual()
        self.last_residual = (None, None)
        while self.time < max_steps:
            self.step(every)
            ru, rT = self.residual()
            self.last_residual = (ru, rT)
            if ru < tol and rT < tol:
                return True
        return False

    def get_state(self):
        """Post-collision populations of the last step, raw FP64, shape [2, 9, ny, nx]."""
        out = self.torch.empty((2, 9, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        _check(lib().lbm_get_state(self.h, out.data_ptr()))
        self.stream.synchronize()
        return out

    def set_state(self, pops):
        t = self.torch.as_tensor(pops, dtype=self.torch.float64, device=self.device).contiguous()
        assert tuple(t.shape) == (2, 9, self.ny, self.nx)
        _check(lib().lbm_set_state(self.h, t.data_ptr()))
        self.stream.synchronize()


class Adjoint:
    """Average Nusselt number of one wall after `steps` steps from the simulation's current
    state, and its gradient with respect to the porosity of every node (discrete adjoint;
    lbm_adjoint_* in include/lbm.h).  The simulation advances by `steps`."""

    def __init__(self, sim: Sim, steps: int, wall: int = 0):
        L = lib()
        torch = sim.torch
        self.sim = sim
        nbytes = int(L.lbm_adjoint_workspace_bytes(sim.h, int(steps)))
        if nbytes == 0:
            raise LbmError(ERR_INVALID, "adjoint workspace size is 0 (invalid steps?)")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=sim.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        h = C.c_void_p()
        nu = C.c_double()
        _check(L.lbm_adjoint_forward(sim.h, int(wall), int(steps), C.c_void_p(aligned), nbytes,
                                     C.byref(h), C.byref(nu)))
        self.h = h
        self.value = nu.value

    def gradient(self, dJ: float = 1.0):
        """dJ * dNu/deps as an FP64 device tensor [ny, nx]."""
        out = self.sim.torch.empty((self.sim.ny, self.sim.nx), dtype=self.sim.torch.float64,
                                   device=self.sim.device)
        _check(lib().lbm_adjoint_backward(self.h, float(dJ), out.data_ptr()))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_adjoint_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _nusselt_function():
    import torch

    class NusseltOfPorosity(torch.autograd.Function):
        """Nu(eps): a fresh simulation of `cfg` with porosity field eps is advanced `steps`
        steps; backward runs the discrete adjoint."""

        @staticmethod
        def forward(ctx, eps, cfg, steps, wall):
            c = dict(cfg, eps_field=eps.detach())
            sim = Sim(c, device=str(eps.device))
            adj = Adjoint(sim, steps, wall)
            ctx.adj = adj
            return torch.tensor(adj.value, dtype=torch.float64, device=eps.device)

        @staticmethod
        def backward(ctx, grad_out):
            g = ctx.adj.gradient(float(grad_out))
            ctx.adj.close()
            return g, None, None, None

    return NusseltOfPorosity


_NusseltFn = None


def nusselt_of_porosity(eps, cfg: dict, steps: int, wall: int = 0):
    """Differentiable average Nusselt number of `wall` after `steps` steps of the problem
    `cfg` with porosity field `eps` (a [ny, nx] FP64 CUDA tensor)."""
    global _NusseltFn
    if _NusseltFn is None:
        _NusseltFn = _nusselt_function()
    return _NusseltFn.apply(eps, cfg, steps, wall)


class Batch:
    """Many problems advanced together (see lbm_batch_* in include/lbm.h)."""

    def __init__(self, cfgs: list, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.cfgs = cfgs
        self.device = torch.device(device)
        L = lib()
        n = len(cfgs)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            keep = []
            arr = (_Params * n)()
            for k, cfg in enumerate(cfgs):
                dev, kk = _device_fields(torch, cfg, self.device, int(cfg["nx"]), int(cfg["ny"]))
                keep += kk
                arr[k] = make_params(cfg, dev)
            nbytes = int(L.lbm_batch_workspace_bytes(arr, n))
            if nbytes == 0:
                for k in range(n):
                    _check(L.lbm_derive(C.byref(arr[k]), C.byref(_Derived())))
                raise LbmError(ERR_INVALID, "batch rejected (mixed storage types?)")
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.workspace.data_ptr() + 255) // 256 * 256
            h = C.c_void_p()
            _check(L.lbm_batch_init(arr, n, C.c_void_p(aligned), nbytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
            self.h = h
            self.stream.synchronize()
            del keep
        self.problems = [Sim._wrap(L.lbm_batch_problem(self.h, k), cfgs[k], self.device, self.stream, self)
                         for k in range(n)]

    def __len__(self):
        return len(self.problems)

    def __getitem__(self, k):
        return self.problems[k]

    def step(self, n: int = 1):
        _check(lib().lbm_batch_step(self.h, int(n)))

    def autotune(self, steps: int = 10):
        """Times the candidate block widths (64, 128, 256 threads) of the launches that run
        under the current steps per pass (the two-step main launch, or the one-step update)
        and keeps the fastest; returns (chosen width, {width: ms per step}).  The problems'
        states are unchanged."""
        w = C.c_int32()
        ms = (C.c_double * 3)()
        _check(lib().lbm_batch_autotune(self.h, int(steps), C.byref(w), ms))
        return w.value, {64: ms[0], 128: ms[1], 256: ms[2]}

    def set_width(self, width: int):
        """Block width (64, 128, 256 threads) of the launches of the current steps per pass."""
        _check(lib().lbm_batch_set_width(self.h, int(width)))

    @property
    def fusion(self) -> int:
        """Time steps per batched pass (1 or 2)."""
        return int(lib().lbm_batch_fusion(self.h))

    @fusion.setter
    def fusion(self, steps_per_pass: int):
        _check(lib().lbm_batch_set_fusion(self.h, int(steps_per_pass)))

    def check(self):
        """Per-problem non-finite flags (numpy int32 array)."""
        flags = (C.c_int32 * len(self.problems))()
        st = lib().lbm_batch_check(self.h, flags)
        if st not in (OK, ERR_NONFINITE):
            _check(st)
        return np.array(flags[:], dtype=np.int32)

    def close(self):
        if getattr(self, "h", None):
            for p in self.problems:
                p.h = None
            lib().lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
