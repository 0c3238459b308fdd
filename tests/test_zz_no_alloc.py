"""lbm_residual_noalloc, the entry point for callers that cannot allocate: its reduction
scratch is the library's static device array instead of the context's workspace.  Checked
through the C interface against lbm_residual on the same states (bitwise: the same kernels
run in the same order), on two calls in a row with the second on a smaller grid, and
interleaved with lbm_residual on one context (they share the snapshot)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_02976_amd import lbm
    lbm.lib()
    return lbm


def _call(gpu, fn, sim):
    ru, rT = C.c_double(), C.c_double()
    st = getattr(gpu.lib(), fn)(sim.h, C.byref(ru), C.byref(rT))
    assert st == 0, (fn, st, gpu.lib().lbm_last_error())
    return ru.value, rT.value


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_residual_equals_workspace_residual(gpu, storage):
    # the second grid is smaller than the first: the static array keeps the first call's
    # partial sums beyond the second grid's, which the second call must not read
    for nx, ny, seed in ((301, 203, 3), (37, 29, 4)):
        _say(f"case: {storage} random case {nx} x {ny} (seed {seed}), residual vs residual_noalloc")
        cfg = W.random_case(seed, nx, ny, storage=storage, eps_field=True)
        a, b = gpu.Sim(cfg), gpu.Sim(cfg)
        for it in range(3):
            ra = _call(gpu, "lbm_residual", a)
            rb = _call(gpu, "lbm_residual_noalloc", b)
            _say(f"  call {it}: {ra} / {rb}")
            assert ra == rb, (it, ra, rb)
            if it == 0:
                assert ra == (-1.0, -1.0)
            else:
                assert ra[0] > 0 and ra[1] > 0
            a.step(50)
            b.step(50)
        a.close()
        b.close()


def test_noalloc_and_workspace_residual_share_the_snapshot(gpu):
    cfg = W.random_case(5, 64, 40, storage="f64")
    a, b = gpu.Sim(cfg), gpu.Sim(cfg)
    _say("case: f64 random case 64 x 40, alternating entry points on one context")
    seq = ("lbm_residual", "lbm_residual_noalloc", "lbm_residual", "lbm_residual_noalloc")
    for it, fn in enumerate(seq):
        ra = _call(gpu, fn, a)
        rb = _call(gpu, "lbm_residual", b)
        assert ra == rb, (it, fn, ra, rb)
        a.step(20)
        b.step(20)


def test_noalloc_residual_rejects_grids_beyond_the_scratch(gpu):
    """A 5200 x 5200 grid needs 105,707 partial sums of 40 bytes, more than the 4 MiB array
    holds: a clear error, while lbm_residual still works on it."""
    cfg = W.cavity(5200, storage="f16")
    cfg["T_init"] = None
    _say("case: f16 cavity 5200 x 5200, residual_noalloc beyond the static scratch")
    sim = gpu.Sim(cfg)
    ru, rT = C.c_double(), C.c_double()
    st = gpu.lib().lbm_residual_noalloc(sim.h, C.byref(ru), C.byref(rT))
    msg = gpu.lib().lbm_last_error()
    msg = msg.decode() if isinstance(msg, bytes) else str(msg)
    _say(f"  status {st}: {msg}")
    assert st == 1 and "static scratch" in msg
    assert sim.residual() == (None, None)
    sim.close()
