"""Host-side checks of the C interface (no GPU work): the library loads, exports every
function declared in include/lbm.h, and validates parameters exactly as documented;
the lattice constants it derives agree with the oracle's independent derivation."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lbm():
    from paper_1505_02976_amd import lbm as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1505_02976_amd import build
        build.build()
    return L


def _declared():
    with open(os.path.join(ROOT, "include", "lbm.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lbm):
    lib = C.CDLL(lbm.LIB_PATH)
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(lbm.EXPORTS) == set(names)


def test_struct_sizes_match_header(lbm):
    # lbm_wall: 2 doubles, 2 int32, 2 doubles; lbm_params ends on two int32
    assert C.sizeof(lbm._Wall) == 40
    assert C.sizeof(lbm._Params) == 4 * 4 + 4 * 40 + 18 * 8 + 5 * 8 + 8


@pytest.mark.parametrize("cfg", [W.cavity(128), W.channel(), W.large_cavity(),
                                 W.random_case(3, 40, 30), W.random_case(4, 17, 9, periodic_x=1)],
                         ids=["cavity", "channel", "large", "rand3", "rand4"])
def test_derived_constants_match_oracle(lbm, oracle_mod, cfg):
    a = lbm.derived(cfg)
    b = oracle_mod.derived(cfg)
    for k in a:
        assert math.isclose(a[k], b[k], rel_tol=1e-14, abs_tol=1e-300), k


def _bad(**kw):
    cfg = W.cavity(32)
    cfg.update(kw)
    return cfg


@pytest.mark.parametrize("cfg,msg", [
    (_bad(tau_f=0.5), "tau_f"),
    (_bad(A=0.6, B=0.0), "nu_e"),
    (_bad(A=0.0, B=0.5), "alpha_e"),
    (_bad(eps=0.0), "eps"),
    (_bad(eps=1.2), "eps"),
    (_bad(Da=0.0), "Da"),
    (_bad(Ra=0.0), "Ra"),
    (_bad(nx=2), "needs"),
    (_bad(ny=3), "needs"),          # Neumann walls on y need 4 nodes
    (_bad(storage="f64", sigma=-1.0), "sigma"),
])
def test_invalid_parameters_are_rejected(lbm, cfg, msg):
    with pytest.raises(lbm.LbmError) as ei:
        lbm.derived(cfg)
    assert ei.value.status == lbm.ERR_INVALID
    assert msg in str(ei.value)
    assert lbm.workspace_bytes(cfg) == 0


def test_workspace_size_scales_with_storage(lbm):
    sizes = {s: lbm.workspace_bytes(W.large_cavity(storage=s)) for s in ("f64", "f32", "f16")}
    N = 4096 * 4096
    # two buffers of 18 planes plus the FP64 residual snapshot (3 fields)
    for s, es in (("f64", 8), ("f32", 4), ("f16", 2)):
        # tiles of 62 columns pad 4096 to 4154 (1.4 %)
        assert 2 * 18 * N * es + 24 * N <= sizes[s] < 1.03 * (2 * 18 * N * es + 24 * N) + 2 ** 20


def test_init_rejects_null_workspace(lbm):
    prm = lbm.make_params(W.cavity(32))
    h = C.c_void_p()
    st = lbm.lib().lbm_init(C.byref(prm), None, 0, None, C.byref(h))
    assert st == lbm.ERR_INVALID and not h.value


def test_batch_rejects_mixed_storage(lbm):
    cfgs = [W.cavity(32, storage="f32"), W.cavity(40, storage="f64")]
    arr = (lbm._Params * 2)()
    for k, c in enumerate(cfgs):
        arr[k] = lbm.make_params(c)
    assert lbm.lib().lbm_batch_workspace_bytes(arr, 2) == 0
    assert "storage" in lbm.lib().lbm_last_error().decode()
    cfgs[1]["storage"] = "f32"
    arr[1] = lbm.make_params(cfgs[1])
    single = lbm.workspace_bytes(cfgs[0]) + lbm.workspace_bytes(cfgs[1])
    assert lbm.lib().lbm_batch_workspace_bytes(arr, 2) >= single


def test_batch_error_names_problem_and_reason(lbm):
    # the per-problem message is formatted from the previous message: it must come through intact
    cfgs = [W.cavity(32, storage="f32"), W.cavity(40, storage="f32")]
    arr = (lbm._Params * 2)()
    for k, c in enumerate(cfgs):
        arr[k] = lbm.make_params(c)
    arr[1].tau_f = 0.5
    assert lbm.lib().lbm_batch_workspace_bytes(arr, 2) == 0
    assert lbm.lib().lbm_last_error().decode() == "problem 1: tau_f and tau_T must exceed 1/2"


def test_one_hip_runtime_whatever_the_import_order():
    # loading the library before torch must not bring a second HIP/HSA runtime into the process
    code = ("from paper_1505_02976_amd import lbm; lbm.lib(); import torch; "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') "
            "if 'libamdhip64' in l or 'libhsa-runtime64' in l}))")
    import subprocess, sys
    out = subprocess.run([sys.executable, "-c", code], cwd=os.path.dirname(os.path.dirname(__file__)),
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert sum("libamdhip64" in p for p in libs) == 1, libs
    assert sum("libhsa-runtime64" in p for p in libs) == 1, libs


def test_exports_every_declared_3d_symbol(lbm):
    with open(os.path.join(ROOT, "include", "lbm3d.h")) as fh:
        names = sorted(set(re.findall(r"\b(lbm3_[a-z_]+)\s*\(", fh.read())))
    assert len(names) == 9, names
    lib = C.CDLL(lbm.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_3d_struct_sizes_and_validation(lbm):
    import workloads as W
    from paper_1505_02976_amd import lbm3d as L3
    # lbm3_wall: 3 doubles, 2 int32, 2 doubles; lbm3_params: 6 int32, 6 walls, 19 doubles, 2 int32, 3 pointers
    assert C.sizeof(L3._Wall3) == 48
    assert C.sizeof(L3._Params3) == 24 + 6 * 48 + 19 * 8 + 8 + 24
    cfg = W.layer3d(16, 8, 12)
    n = 16 * 8 * 12
    assert L3.workspace_bytes(cfg) == 2 * ((2 * 19 * n * 8 + 255) // 256 * 256) + 256
    assert L3.workspace_bytes(dict(cfg, storage="f32")) == 2 * ((2 * 19 * n * 4 + 255) // 256 * 256) + 256
    assert L3.workspace_bytes(dict(cfg, nz=3)) == 0
    assert "nz >= 4" in lbm.lib().lbm_last_error().decode()
    assert L3.workspace_bytes(dict(cfg, nz=3, periodic_z=1)) > 0
    assert L3.workspace_bytes(dict(cfg, nx=3, periodic_x=0)) == 0
    assert "nx >= 4" in lbm.lib().lbm_last_error().decode()
    assert L3.workspace_bytes(dict(cfg, nx=4, periodic_x=0, walls=cfg["walls"] + [{}, {}])) > 0
    assert L3.workspace_bytes(dict(cfg, ny=3, periodic_y=0)) == 0
    assert "ny >= 4" in lbm.lib().lbm_last_error().decode()
    assert L3.workspace_bytes(dict(cfg, tau_f=0.5)) == 0
    assert L3.workspace_bytes(dict(cfg, A=0.6, B=0.1)) == 0
    assert "nu_e" in lbm.lib().lbm_last_error().decode()
    c = L3.lattice()
    assert len(set(c)) == 19 and (0, 0, 0) in c
    assert sorted(sum(abs(v) for v in ci) for ci in c) == [0] + [1] * 6 + [2] * 12


def test_null_handles_are_rejected_without_touching_the_device(lbm):
    """Every entry point that takes a handle returns LBM_ERR_INVALID for a NULL one, with a
    message, and never reaches the device (these calls run without a GPU)."""
    lib = C.CDLL(lbm.LIB_PATH)
    lib.lbm_last_error.restype = C.c_char_p
    d = C.c_double()
    two = (C.c_double * 2)()
    calls = {
        "lbm_step": lambda: lib.lbm_step(None, C.c_int64(5)),
        "lbm_set_check_interval": lambda: lib.lbm_set_check_interval(None, C.c_int64(10)),
        "lbm_set_fusion": lambda: lib.lbm_set_fusion(None, C.c_int32(2)),
        "lbm_nusselt": lambda: lib.lbm_nusselt(None, C.c_int32(0), C.byref(d)),
        "lbm_residual": lambda: lib.lbm_residual(None, C.byref(two, 0), C.byref(two, 8)),
        "lbm_residual_noalloc": lambda: lib.lbm_residual_noalloc(None, C.byref(two, 0), C.byref(two, 8)),
        "lbm_batch_step": lambda: lib.lbm_batch_step(None, C.c_int64(2)),
        "lbm_batch_set_fusion": lambda: lib.lbm_batch_set_fusion(None, C.c_int32(1)),
        "lbm_adjoint_backward": lambda: lib.lbm_adjoint_backward(None, C.c_double(1.0), None),
        "lbm3_step": lambda: lib.lbm3_step(None, C.c_int64(1)),
        "lbm3_nusselt": lambda: lib.lbm3_nusselt(None, C.c_int32(0), C.byref(d)),
    }
    for name, call in calls.items():
        assert call() == lbm.ERR_INVALID, name
        assert lib.lbm_last_error(), name
    # handle-less destructors accept NULL
    lib.lbm_destroy(None)
    lib.lbm_batch_destroy(None)
    lib.lbm_adjoint_destroy(None)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits with status 2 and says why,
    before touching torch or the library."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "8"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "asked for 8" in r.stderr
    assert r.stdout == ""
