"""Batched stepping of many problems (the same launches per step, or per two-step pass,
for all problems: two-step passes on two streams, one-step updates replayed from a HIP graph
of 64 steps) against the single-problem path and the oracle.  Graph replays are
interleaved with eager work and synchronisations, and every replay is checked."""
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


def _cases(storage):
    return [
        W.random_case(21, 40, 30, storage=storage),
        W.random_case(22, 17, 90, storage=storage, moving_walls=True),
        W.random_case(23, 128, 64, storage=storage, with_Q=True),
        W.random_case(24, 33, 33, periodic_x=1, storage=storage),
        W.random_case(25, 64, 64, storage=storage, eps_field=True),
        W.cavity(96, storage=storage),
    ]


def test_batch_fp64_matches_single_and_oracle(gpu, oracle_mod):
    import torch
    cfgs = _cases("f64")
    _say(f"case: batch of {len(cfgs)} FP64 problems, 64 + 64 + 7 steps")
    batch = gpu.Batch(cfgs)
    singles = [gpu.Sim(c) for c in cfgs]
    for chunk in (64, 64, 7):
        batch.step(chunk)
        # eager work on the same stream between replays
        _ = batch[2].fields()
        for s in singles:
            s.step(chunk)
        torch.cuda.synchronize()
        for k, s in enumerate(singles):
            a = batch[k].get_state()
            b = s.get_state()
            assert bool((a == b).all()), (k, chunk, float((a - b).abs().max()))
        assert all(p.time == batch[0].time for p in batch.problems)
    for k, cfg in enumerate(cfgs):
        ref = oracle_mod.Oracle(cfg)
        ref.step(135)
        f, g = ref.populations(post=True)
        st = batch[k].get_state().cpu().numpy()
        d = max(float(np.abs(st[0] - f).max()), float(np.abs(st[1] - g).max()))
        assert d < 1e-10, (k, d)
    assert not batch.check().any()


def test_batch_fp32_bitwise_equals_single(gpu):
    cfgs = W.ensemble(count=6, side_lo=32, side_hi=80, storage="f32", max_cell_re=5.0)
    _say("case: ensemble of 6 FP32 cavities, 200 steps")
    batch = gpu.Batch(cfgs)
    batch.step(200)
    for k, cfg in enumerate(cfgs):
        s = gpu.Sim(cfg)
        s.step(200)
        assert bool((batch[k].get_state() == s.get_state()).all()), k
        assert abs(batch[k].nusselt(0) - s.nusselt(0)) == 0.0


def test_batch_nonfinite_flags(gpu):
    cfgs = _cases("f32")[:3]
    batch = gpu.Batch(cfgs)
    batch.step(3)
    st = batch[1].get_state()
    st[1, 4, 3, 5] = float("inf")
    batch[1].set_state(st)
    flags = batch.check()
    assert flags.tolist() == [0, 1, 0]


def test_batch_member_cannot_step_alone(gpu):
    batch = gpu.Batch(_cases("f32")[:2])
    with pytest.raises(gpu.LbmError):
        batch[0].step(1)


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_batch_block_widths_and_autotune(gpu, storage):
    """Every block width gives bitwise the single-problem result; the autotuner leaves the
    states untouched and keeps one of the candidates."""
    import torch
    cfgs = _cases(storage)
    _say(f"case: batch of {len(cfgs)} {storage} problems, widths 64/128/256 and autotune")
    singles = [gpu.Sim(c) for c in cfgs]
    for s in singles:
        s.step(70)
    for width in (64, 128, 256):
        batch = gpu.Batch(cfgs)
        batch.set_width(width)
        batch.step(70)          # FP16: one graph replay and 6 single steps; else 35 passes
        torch.cuda.synchronize()
        for k, s in enumerate(singles):
            assert bool((batch[k].get_state() == s.get_state()).all()), (width, k)
        batch.close()
    batch = gpu.Batch(cfgs)
    batch.step(5)
    before = [p.get_state() for p in batch.problems]
    w, ms = batch.autotune(4)
    _say(f"  autotune: chose {w}, ms/step {ms}")
    assert w in (64, 128, 256) and all(v > 0 for v in ms.values())
    for k, p in enumerate(batch.problems):
        assert bool((p.get_state() == before[k]).all()), k
    batch.step(65)
    for k, s in enumerate(singles):
        assert bool((batch[k].get_state() == s.get_state()).all()), ("tuned", k)
    with pytest.raises(gpu.LbmError):
        batch.set_width(96)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_two_step_passes_bitwise(gpu, storage):
    """Two-step batched passes, odd step counts and a switch to one step per pass (graph
    replays, realigned after odd counts) and back all give bitwise the single-problem
    states."""
    import torch
    cfgs = _cases(storage) + [W.random_case(26, 4, 8, storage=storage),
                              W.random_case(27, 70, 8, periodic_x=1, storage=storage)]
    _say(f"case: batch of {len(cfgs)} {storage} problems, two-step passes, chunks 1/65/64/3/130")
    batch = gpu.Batch(cfgs)
    assert batch.fusion == 2
    singles = [gpu.Sim(c) for c in cfgs]
    total = 0
    for chunk, fuse in ((1, 2), (65, 2), (64, 2), (3, 2), (130, 2), (66, 1), (64, 2)):
        batch.fusion = fuse
        batch.step(chunk)
        _ = batch[0].fields()
        for s in singles:
            s.step(chunk)
        total += chunk
        torch.cuda.synchronize()
        for k, s in enumerate(singles):
            a, b = batch[k].get_state(), s.get_state()
            assert bool((a == b).all()), (chunk, fuse, k, float((a - b).abs().max()))
        assert batch[0].time == total
    assert not batch.check().any()


def test_batch_fp16_has_one_step_passes(gpu):
    batch = gpu.Batch(_cases("f16")[:2])
    assert batch.fusion == 1
    with pytest.raises(gpu.LbmError):
        batch.fusion = 2
