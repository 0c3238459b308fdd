"""Parity of the HIP path (through the C interface) with the oracle, element by element.

FP64 storage must agree with the oracle to max-abs 1e-10 on populations and on every
macroscopic field; FP32 storage to relative L2 1e-5 on u and T; FP16 storage errors are
measured and bounded loosely (they are reported, not targeted).  Inputs are seeded and
synthetic; see workloads.py.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("p", "ux", "uy", "T", "Sxx", "Sxy", "Syy", "dTdx", "dTdy")


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


def _compare(sim, ref, tol, pops=True):
    g = sim.fields()
    o = ref.fields()
    worst = {}
    for k in FIELDS:
        worst[k] = float(np.max(np.abs(g[k].cpu().numpy() - o[k])))
    if pops:
        st = sim.get_state().cpu().numpy()
        f, gg = ref.populations(post=True)
        worst["f"] = float(np.max(np.abs(st[0] - f)))
        worst["g"] = float(np.max(np.abs(st[1] - gg)))
    bad = {k: v for k, v in worst.items() if not v <= tol}
    assert not bad, worst
    return worst


def test_cavity_fp64_1000_steps(gpu, oracle_mod):
    cfg = W.cavity(128, storage="f64")
    _say("case: cavity 128x128 eps 0.6 Da 1e-2 Ra 1e5 FP64, 1000 steps")
    sim = gpu.Sim(cfg)
    sim.step(1000)
    ref = oracle_mod.Oracle(cfg)
    ref.step(1000)
    w = _compare(sim, ref, 1e-10)
    _say(f"  worst {w}")
    # Nusselt numbers and the residual use the same fixed definitions on both sides
    for wall in (0, 1, 2, 3):
        assert abs(sim.nusselt(wall) - ref.nusselt(wall)) < 1e-10


@pytest.mark.parametrize("seed,nx,ny,px,py,extra", [
    (1, 133, 77, 0, 0, {}),
    (2, 257, 5, 1, 0, {"moving_walls": True}),
    (3, 97, 45, 1, 1, {"with_Q": True}),
    (4, 64, 300, 0, 1, {"eps_field": True}),
    (5, 300, 64, 0, 0, {"eps_field": True, "with_Q": True, "moving_walls": True}),
    (6, 4, 4, 0, 0, {}),
    (7, 1, 33, 1, 0, {}),
])
def test_random_cases_fp64(gpu, oracle_mod, seed, nx, ny, px, py, extra):
    cfg = W.random_case(seed, nx, ny, periodic_x=px, periodic_y=py, storage="f64", **extra)
    if nx == 4 and ny == 4:
        for w in cfg["walls"]:
            w["kind"] = "T"            # 4 nodes suffice for Neumann; keep one all-Dirichlet box
    _say(f"case: random seed {seed} {nx}x{ny} periodic ({px},{py}) {extra} FP64, 0 and 40 steps")
    sim = gpu.Sim(cfg)
    ref = oracle_mod.Oracle(cfg)
    _compare(sim, ref, 1e-12)
    sim.step(40)
    ref.step(40)
    w = _compare(sim, ref, 1e-10)
    _say(f"  worst {w}")


def test_channel_fp64_steady(gpu, oracle_mod):
    cfg = W.channel(storage="f64")
    _say("case: porous channel 4x64 FP64 to residual 1e-10")
    sim = gpu.Sim(cfg)
    assert sim.run_to_steady(1e-10, 50000)
    ref = oracle_mod.Oracle(cfg)
    ref.step(sim.time)
    _compare(sim, ref, 1e-10)
    ru, rT = sim.residual()
    assert ru < 1e-10 and rT < 1e-10


def test_residual_matches_oracle(gpu, oracle_mod):
    cfg = W.cavity(64, storage="f64")
    sim = gpu.Sim(cfg)
    ref = oracle_mod.Oracle(cfg)
    assert sim.residual() == (None, None)
    ref.residual()
    for _ in range(3):
        sim.step(100)
        ref.step(100)
        a = sim.residual()
        b = ref.residual()
        assert abs(a[0] - b[0]) < 1e-10 * max(1.0, b[0]) and abs(a[1] - b[1]) < 1e-10 * max(1.0, b[1])


def test_fp64_is_deterministic(gpu):
    cfg = W.random_case(9, 150, 70, storage="f64", eps_field=True)
    a = gpu.Sim(cfg)
    b = gpu.Sim(cfg)
    a.step(25)
    b.step(25)
    assert bool((a.get_state() == b.get_state()).all())


def _rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def test_cavity_fp32_and_fp16_errors(gpu, oracle_mod):
    ref = oracle_mod.Oracle(W.cavity(128))
    ref.step(1000)
    o = ref.fields()
    errs = {}
    for storage in ("f32", "f16"):
        _say(f"case: cavity 128x128 {storage}, 1000 steps")
        sim = gpu.Sim(W.cavity(128, storage=storage))
        sim.step(1000)
        g = sim.fields()
        errs[storage] = {k: _rel_l2(g[k].cpu().numpy(), o[k]) for k in ("ux", "uy", "T")}
        errs[storage]["Nu"] = abs(sim.nusselt(0) - ref.nusselt(0))
    _say(f"  rel L2 errors vs FP64 oracle: {errs}")
    assert max(errs["f32"][k] for k in ("ux", "uy", "T")) < 1e-5
    assert errs["f32"]["Nu"] < 1e-4
    assert max(errs["f16"][k] for k in ("ux", "uy", "T")) < 5e-2


def test_nonfinite_is_detected(gpu):
    import torch
    cfg = W.cavity(32, storage="f32")
    sim = gpu.Sim(cfg)
    sim.step(3)
    st = sim.get_state()
    st[0, 0, 10, 10] = float("nan")   # rest population: never streamed, still detected
    sim.set_state(st)
    with pytest.raises(gpu.NonFiniteError):
        sim.residual()
    torch.cuda.synchronize()


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_step_checks_for_nonfinite_populations(gpu, storage):
    """With a check interval, lbm_step stops with LBM_ERR_NONFINITE at the first multiple of
    the interval after a population turned infinite; without one it stays asynchronous."""
    cfg = W.random_case(9, 40, 30, storage=storage)
    sim = gpu.Sim(cfg)
    sim.set_check_interval(100)
    sim.step(250)                      # checks at 100 and 200 pass
    assert sim.time == 250
    st = sim.get_state()
    st[1, 3, 10, 7] = float("inf")
    sim.set_state(st)
    with pytest.raises(gpu.NonFiniteError):
        sim.step(300)
    assert sim.time == 300              # stopped at the check, the later steps not enqueued
    sim.set_check_interval(0)
    sim.step(7)                         # no check, no error
    assert sim.time == 307


def test_get_set_state_roundtrip(gpu):
    for storage, tol in (("f64", 0.0), ("f32", 1e-7), ("f16", 1e-4)):
        cfg = W.random_case(12, 45, 31, storage=storage)
        sim = gpu.Sim(cfg)
        sim.step(5)
        st = sim.get_state()
        sim.set_state(st)
        st2 = sim.get_state()
        assert float((st - st2).abs().max()) <= tol


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 2e-6), ("f16", 5e-3)])
def test_full_size_cavity(gpu, oracle_mod, storage, tol):
    """The 4096 x 4096 throughput workload in the launch configuration bench.py times,
    started from smooth random pressure and velocity fields so that every term of the
    step is active at every node; three steps against the oracle on the whole grid.
    FP64: max-abs on all fields; FP32/FP16: relative L2 of u, T and p."""
    n = 4096
    cfg = W.large_cavity(n, storage=storage)
    rng = np.random.default_rng(42)
    cfg["p_init"] = W.smooth_field(n, n, rng, 1e-3)
    cfg["ux_init"] = W.smooth_field(n, n, rng, 0.02)
    cfg["uy_init"] = W.smooth_field(n, n, rng, 0.02)
    _say(f"case: full-size cavity {n}x{n} {storage}, 3 steps")
    sim = gpu.Sim(cfg)
    sim.step(3)
    g = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    del sim
    ref = oracle_mod.Oracle(cfg)
    ref.step(3)
    o = ref.fields()
    if storage == "f64":
        worst = {k: float(np.max(np.abs(g[k] - o[k]))) for k in FIELDS}
        _say(f"  worst {worst}")
        assert max(worst.values()) < tol, worst
    else:
        errs = {k: _rel_l2(g[k], o[k]) for k in ("ux", "uy", "T", "p")}
        _say(f"  rel L2 {errs}")
        assert max(errs.values()) < tol, errs


def test_degenerate_step_counts(gpu):
    """Zero steps leave the state and the time untouched (single problem, batch, with and
    without a check interval); negative counts and intervals are rejected with
    LBM_ERR_INVALID and change nothing."""
    import torch
    for storage in ("f64", "f32", "f16"):
        cfg = W.random_case(31, 40, 24, storage=storage)
        sim = gpu.Sim(cfg)
        sim.step(3)
        before = sim.get_state()
        sim.step(0)
        sim.set_check_interval(7)
        sim.step(0)
        with pytest.raises(gpu.LbmError):
            sim.step(-1)
        with pytest.raises(gpu.LbmError):
            sim.set_check_interval(-2)
        torch.cuda.synchronize()
        assert sim.time == 3
        assert bool((sim.get_state() == before).all()), storage
        batch = gpu.Batch([cfg, W.random_case(32, 17, 9, storage=storage)])
        batch.step(2)
        snap = [p.get_state() for p in batch.problems]
        batch.step(0)
        with pytest.raises(gpu.LbmError):
            batch.step(-3)
        torch.cuda.synchronize()
        assert batch[0].time == 2
        for k, p in enumerate(batch.problems):
            assert bool((p.get_state() == snap[k]).all()), (storage, k)
        batch.close()
