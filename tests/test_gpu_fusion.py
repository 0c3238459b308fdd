"""The two-step pass against single steps, bit for bit: every node update of the pass is
the one-step node code with the same inputs (FP16 storage rounds the intermediate state
to the stored format), so any difference is an indexing, shift or boundary error.  Grids
cover all wall combinations and the three instances of the pass (lean, vertical walls
only, full), ragged sizes (the last column chunk partly past the wall, or, for one or two
leftover columns, overlapping the previous one; periodic grids whose last chunk overlaps
or wraps; a short last row band), porosity fields, moving walls and a heat source, an odd
number of steps (the last one single) and both layouts (planes for FP64, tiles for
FP32/FP16)."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_02976_amd import lbm
    lbm.lib()
    return lbm


CASES = [
    (41, 130, 40, 0, 0, {"eps_field": True, "with_Q": True, "moving_walls": True}),
    (42, 187, 45, 0, 0, {"moving_walls": True}),
    (43, 200, 64, 1, 0, {"with_Q": True, "moving_walls": True}),
    (44, 128, 33, 0, 1, {"eps_field": True}),
    (45, 150, 70, 1, 1, {"with_Q": True}),
    (46, 311, 97, 0, 0, {"eps_field": True}),
    (47, 124, 32, 0, 0, {}),
    (48, 17, 9, 0, 0, {"moving_walls": True, "with_Q": True}),
    (49, 40, 30, 1, 0, {"eps_field": True}),
    (50, 64, 8, 0, 0, {}),
    (51, 5, 12, 0, 1, {}),
    (52, 33, 33, 1, 1, {"with_Q": True}),
    (53, 61, 20, 0, 0, {"eps_field": True, "moving_walls": True}),
    (54, 63, 21, 1, 0, {}),
    (55, 126, 24, 0, 0, {"moving_walls": True}),
    (56, 250, 19, 0, 1, {"eps_field": True}),
]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("seed,nx,ny,px,py,extra", CASES, ids=[f"{c[1]}x{c[2]}-p{c[3]}{c[4]}" for c in CASES])
def test_two_step_pass_is_bitwise_two_steps(gpu, storage, seed, nx, ny, px, py, extra):
    cfg = W.random_case(seed, nx, ny, periodic_x=px, periodic_y=py, storage=storage, **extra)
    a = gpu.Sim(cfg)
    b = gpu.Sim(cfg)
    assert a.fusion == (1 if storage == "f16" else 2)
    a.fusion = 2
    b.fusion = 1
    for n in (2, 7, 30):
        a.step(n)
        b.step(n)
        sa, sb = a.get_state(), b.get_state()
        assert bool((sa == sb).all()), (n, float((sa - sb).abs().max()))
    assert a.time == b.time == 39
    if not py:
        assert a.nusselt(2) == b.nusselt(2)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_two_step_pass_full_width(gpu, storage):
    """The bench's grid width with walls in x (67 column chunks of 62, the last one four
    columns wide) and a porosity field: passes equal single steps bit for bit."""
    cfg = W.random_case(57, 4096, 264, storage=storage, eps_field=True, moving_walls=True)
    print(f"case: {storage} 4096x264 walled, 9 steps", flush=True)
    a = gpu.Sim(cfg)
    b = gpu.Sim(cfg)
    b.fusion = 1
    a.step(9)
    b.step(9)
    sa, sb = a.get_state(), b.get_state()
    assert bool((sa == sb).all()), float((sa - sb).abs().max())


def test_fusion_setting(gpu):
    small = gpu.Sim(W.random_case(48, 100, 7))
    assert small.fusion == 1
    with pytest.raises(gpu.LbmError):
        small.fusion = 2
    with pytest.raises(gpu.LbmError):
        small.fusion = 3
    big = gpu.Sim(W.cavity(128, storage="f64"))
    assert big.fusion == 2
    big.fusion = 1
    assert big.fusion == 1
    assert gpu.Sim(W.cavity(128, storage="f32")).fusion == 2
    assert gpu.Sim(W.cavity(128, storage="f16")).fusion == 1


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_timed_steps_equal_plain_steps(gpu, storage):
    """lbm_step_timed advances exactly as lbm_step (the events it brackets passes with do
    not change the work), over repeated calls that reuse the context's timing events,
    with an odd count (a two-step schedule's last step single) and a count spanning more
    than one group of read-back events; it reports positive launch times, the main
    launch's node count and the steps per pass."""
    cfg = W.random_case(58, 150, 70, storage=storage, moving_walls=True)
    a = gpu.Sim(cfg)
    b = gpu.Sim(cfg)
    per = a.fusion
    for n, every in ((2, 1), (7, 1), (600, 1), (33, 8)):
        main_ms, rest_ms, nodes, k = a.step_timed(n, every)
        b.step(n)
        assert k == per
        assert main_ms > 0.0 and rest_ms >= 0.0
        assert 0 < nodes <= cfg["nx"] * cfg["ny"]
        sa, sb = a.get_state(), b.get_state()
        assert bool((sa == sb).all()), (n, float((sa - sb).abs().max()))
    assert a.time == b.time == 642
