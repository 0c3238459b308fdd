"""Parity at the largest sizes one GPU holds comfortably, by a property that holds at any
size: a problem whose initial fields repeat with period P in a periodic direction stays
P-periodic, so every P-wide tile of a huge grid must equal, bit for bit, the same problem
on a grid one period wide (same kernels, same arithmetic per node), and that small problem
is checked against the oracle.  Element indices exceed 2^32 here (FP16 at 16384 x 16384:
18 x 2^28 populations per buffer), so 32-bit index arithmetic anywhere would show."""
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


def _tile(cfg, reps_y, reps_x):
    big = dict(cfg)
    big["nx"], big["ny"] = cfg["nx"] * reps_x, cfg["ny"] * reps_y
    for k in ("T_init", "p_init", "ux_init", "uy_init", "eps_field"):
        if cfg.get(k) is not None:
            big[k] = np.tile(cfg[k], (reps_y, reps_x))
    return big


def _check_tiles(torch, big_state, small_state, reps_y, reps_x):
    _, _, ny, nx = small_state.shape
    v = big_state.view(2, 9, reps_y, ny, reps_x, nx)
    ref = small_state.view(2, 9, 1, ny, 1, nx)
    return bool((v == ref).all())


@pytest.mark.parametrize("storage,shape,period,px,py", [
    ("f16", (16384, 16384), (64, 64), 1, 1),
    ("f32", (4096, 65536), (4096, 64), 1, 0),
], ids=["f16-periodic-16384x16384", "f32-channel-65536x4096"])
def test_periodic_replication(gpu, oracle_mod, storage, shape, period, px, py):
    import torch
    ny, nx = shape
    pny, pnx = period
    small = W.random_case(31, pnx, pny, periodic_x=px, periodic_y=py, storage=storage,
                          eps_field=True, with_Q=True, moving_walls=not py)
    steps = 4
    _say(f"case: {storage} {nx}x{ny} from {pnx}x{pny} tiles (periodic {px},{py}), {steps} steps")
    s = gpu.Sim(small)
    s.step(steps)
    small_state = s.get_state()
    ref = oracle_mod.Oracle(small)
    ref.step(steps)
    f, g = ref.populations(post=True)
    st = small_state.cpu().numpy()
    rel = max(float(np.abs(st[0] - f).max()), float(np.abs(st[1] - g).max()))
    _say(f"  one period vs oracle: max-abs population difference {rel:.2e}")
    # FP16 keeps 11 significant bits of deviations up to about 0.1 here
    assert rel < (5e-4 if storage == "f16" else 1e-6)
    big = _tile(small, ny // pny, nx // pnx)
    b = gpu.Sim(big)
    del big
    b.step(steps)
    big_state = b.get_state()
    del b
    torch.cuda.synchronize()
    ok = _check_tiles(torch, big_state, small_state, ny // pny, nx // pnx)
    _say(f"  every tile bitwise equal to the one-period run: {ok}")
    assert ok
    del big_state
    torch.cuda.empty_cache()
