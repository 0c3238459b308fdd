"""Throughput benchmark of the fused porous thermal lattice-BGK step on one MI355X.

Workload: natural convection in a 4096 x 4096 porous cavity (eps 0.4, Da 1e-4, Ra 1e7,
Pr 0.71, tau = 1, A and B from Ma = 0.1), FP32 population storage.  One "step" is one
full time step of the method on the whole grid: streaming, boundary scheme, moments,
drag solve, shear rate, temperature gradient, equilibria, collision (all nodes).

Prints one JSON line: MLUPS (million node updates of the coupled flow + temperature
populations per second), the roofline of the dominant kernel (for FP32 and FP64 storage
the two-step pass, whose lean launch k_step2 updates the nodes away from walls by two
time steps per read and write of their populations; for FP16 the one-step interior
launch k_step_bulk), the other storage precisions on the same workload, the one-step
schedule for comparison, the batched ensemble, the adjoint, the Nusselt-number accuracy
of each precision on the 128 x 128 cavity against the FP64 path, and the FP64 CPU oracle
timed on the host as a baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ELEM = {"f64": 8, "f32": 4, "f16": 2}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# the sources the step kernels are compiled from
BULK_SOURCES = ("lbm_device.h", "lbm_kernels.h", "lbm_kernels.hip", "lbm_step2.hip")


def measured_traffic(kernel, storage, n):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, if it
    was taken on this workload and on the kernel sources as they are now (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{storage}_cavity{n}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if kernel_sources_hash() != rec.get("csrc_sha256"):
        return None
    return rec["traffic_bytes_per_launch"]


def kernel_sources_hash():
    """SHA-256 of the kernel sources with comments and blank lines removed (a change of
    wording in a comment does not make the recorded counters stale)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1505_02976_amd", "csrc")
    lines = []
    for p in BULK_SOURCES:
        with open(os.path.join(csrc, p)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


WARMUP_S = 0.5     # minimum wall time of the untimed warm-up (clocks and caches settle)


def warm(sim, warmup, min_s=WARMUP_S):
    """`warmup` untimed steps, then more untimed steps until at least min_s of wall time has
    passed, so that a short --warmup still starts the timed region at steady clocks.  The
    last two go through step_timed, which creates the timing events outside the timed
    region.  Returns (steps, seconds) of the warm-up."""
    t0 = time.perf_counter()
    n = warmup
    sim.step(warmup)
    sim.stream.synchronize()
    chunk = max(2, warmup)
    while time.perf_counter() - t0 < min_s:
        sim.step(chunk)
        sim.stream.synchronize()
        n += chunk
        chunk = min(2 * chunk, 512)
    sim.step_timed(2)
    sim.stream.synchronize()
    n += 2
    return n, time.perf_counter() - t0


def timed_run(lbm, torch, cfg, warmup, steps, every=8, fusion=None):
    """Warm up (warm), then time `steps` steps with HIP events on the simulation's stream;
    inside that region the launches of every `every`-th pass are bracketed by further
    events, which give the mean launch durations (the events cost a few microseconds per
    bracketed pass, included in the total).  A pass is one step, or two with the two-step
    kernel."""
    sim = lbm.Sim(cfg)
    if fusion is not None:
        sim.fusion = fusion
    warm_steps, warm_s = warm(sim, warmup)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(sim.stream):
        t0.record()
        main_ms, rest_ms, main_nodes, per_pass = sim.step_timed(steps, every)
        t1.record()
    t1.synchronize()
    total_ms = t0.elapsed_time(t1)
    nx, ny = cfg["nx"], cfg["ny"]
    mlups = nx * ny * steps / (total_ms * 1e-3) / 1e6
    es = ELEM[cfg["storage"]]
    # a pass reads and writes every population of the nodes it updates once
    bytes_per_launch = main_nodes * 36 * es
    achieved = bytes_per_launch / (main_ms * 1e-3) / 1e9
    res = {
        "mlups": mlups, "ms_per_step": total_ms / steps, "steps_per_pass": per_pass,
        "main_kernel": "k_step2" if per_pass == 2 else "k_step_bulk",
        # MLUPS x the bytes a one-step-per-pass schedule moves per node update
        "one_step_equivalent_GBps": nx * ny * 36 * es * steps / (total_ms * 1e-3) / 1e9,
        "main_kernel_us": main_ms * 1e3, "rest_us": rest_ms * 1e3,
        "main_nodes": main_nodes, "timed_every": every,
        "main_bytes_per_launch": bytes_per_launch, "main_GBps": achieved,
        "frac": achieved / HBM_PEAK_GBS, "warmup_steps_run": warm_steps, "warmup_s": warm_s,
    }
    del sim
    torch.cuda.synchronize()
    return res


def ensemble_run(lbm, torch, W, count=256, steps=10000, warmup=64, max_cell_re=None):
    """Aggregate throughput of an ensemble of cavities of uneven size and parameters,
    advanced together by the batched kernels (two-step passes).  max_cell_re caps
    Ra per cavity at Pr (max_cell_re (N - 1))^2 (None: Ra log-uniform on [1e3, 1e6] for
    every cavity); cavities that turn non-finite are counted."""
    cfgs = W.ensemble(count=count, seed=0, storage="f32", max_cell_re=max_cell_re)
    nodes = sum(c["nx"] * c["ny"] for c in cfgs)
    b = lbm.Batch(cfgs)
    b.step(warmup)
    width, tune_ms = b.autotune(10)
    log(f"ensemble: autotuner chose block width {width} ({tune_ms} ms/step)")
    b.stream.synchronize()

    def timed(n):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(b.stream):
            t0.record()
            b.step(n)
            t1.record()
        t1.synchronize()
        return t0.elapsed_time(t1)

    fusion = b.fusion
    ms = timed(steps)
    flags = b.check()
    one_step = None
    if fusion == 2:
        # the one-step batched schedule on the same states, for comparison
        b.fusion = 1
        n1 = max(64, steps // 5 // 64 * 64)
        ms1 = timed(n1)
        one_step = {"steps": n1, "mlups": nodes * n1 / (ms1 * 1e-3) / 1e6, "ms_per_step": ms1 / n1}
        b.fusion = fusion
    ra = ("Ra log-uniform on [1e3, min(1e6, Pr (%g (N-1))^2)] (grid cell Reynolds number at most %g)"
          % (max_cell_re, max_cell_re)) if max_cell_re else "Ra log-uniform on [1e3, 1e6]"
    res = {"workload": f"{count} porous cavities, side N ~ U{{64..512}}, {ra}, Da 10^U(-4,-1), "
                       f"eps U(0.4,0.9), Pr 1, FP32 storage, seed 0",
           "nodes": nodes, "steps": steps, "mlups": nodes * steps / (ms * 1e-3) / 1e6,
           "ms_per_step": ms / steps, "GBps_algorithmic": nodes * 144 * steps / (ms * 1e-3) / 1e9,
           "nonfinite_problems": int(flags.sum()),
           "steps_per_pass": fusion, "one_step_per_pass": one_step,
           "block_width": width, "autotune_ms_per_step": {str(k): v for k, v in tune_ms.items()}}
    b.close()
    del b
    torch.cuda.synchronize()
    return res


def adjoint_run(lbm, torch, W, n=256, steps=5000, storage="f32"):
    """Gradient of the hot-wall Nusselt number after `steps` steps with respect to the
    porosity of every node of the 256 x 256 adjoint cavity: time of the forward sweep
    (steps + checkpoints) and of the backward sweep (segment recomputation + adjoint steps)."""
    sim = lbm.Sim(W.adjoint_cavity(n, storage=storage))
    sim.stream.synchronize()
    t0 = time.perf_counter()
    adj = lbm.Adjoint(sim, steps, 0)
    t1 = time.perf_counter()
    g = adj.gradient()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    res = {"workload": f"adjoint cavity {n}x{n} (Ra 1e5, Pr 1, Da 1e-2, porosity field), {steps} steps, "
                       f"{storage} storage, adjoint arithmetic " + ("FP64" if storage == "f64" else "FP32"),
           "Nu": adj.value, "forward_s": t1 - t0, "backward_s": t2 - t1,
           "backward_us_per_step": (t2 - t1) / steps * 1e6,
           "backward_node_steps_per_s": n * n * steps / (t2 - t1),
           "grad_l2": float(torch.linalg.vector_norm(g))}
    adj.close()
    del sim
    torch.cuda.synchronize()
    return res


def three_d_run(torch, W, shape=(192, 192, 96), steps=200, warmup=20):
    """The 3-D (D3Q19) path on a porous layer heated from below (Ra 1e4, Da 1e-2, eps 0.6),
    FP64, FP32 and FP16 storage: per step one launch over the interior and one over the wall
    planes, each node reading and writing 2 x 19 populations, timed with events on the
    stream the launches go to."""
    from paper_1505_02976_amd import lbm3d
    nx, ny, nz = shape
    nodes = nx * ny * nz
    out = {"workload": f"porous layer heated from below {nx}x{ny}x{nz}, Ra 1e4, Da 1e-2, eps 0.6, D3Q19",
           "nodes": nodes}
    for storage, es in (("f64", 8), ("f32", 4), ("f16", 2)):
        sim = lbm3d.Sim3(W.layer3d(nx, ny, nz, Ra=1e4, Da=1e-2, storage=storage))
        sim.step(warmup)
        st = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.synchronize()
        a.record(st)
        sim.step(steps)
        b.record(st)
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        bytes_step = nodes * 2 * 38 * es
        out[storage] = {"mlups": nodes / (ms * 1e3), "ms_per_step": ms, "bytes_per_step": bytes_step,
                        "GBps": bytes_step / (ms * 1e6), "frac": bytes_step / (ms * 1e6) / HBM_PEAK_GBS}
        sim.close()
        del sim
    return out


def accuracy(lbm, W, n=128, tol=1e-9, max_steps=600000):
    """Average Nusselt number of the hot wall on the n x n cavity per precision: FP64 run
    until both residuals of Sec. 4 fall below tol (or max_steps), FP32 and FP16 storage the
    same number of steps, each compared with FP64 at that state."""
    out = {}
    steps = None
    converged, reached = None, None
    for storage in ("f64", "f32", "f16"):
        sim = lbm.Sim(W.cavity(n, storage=storage))
        if storage == "f64":
            converged = sim.run_to_steady(tol, max_steps)
            reached = sim.last_residual
            steps = sim.time
            log(f"accuracy f64: residuals {reached} after {steps} steps (converged: {converged})")
        else:
            sim.step(steps)
        out[storage] = {"Nu": sim.nusselt(0), "steps": sim.time}
        log(f"accuracy {storage}: Nu = {out[storage]['Nu']:.6f} after {sim.time} steps")
    ref = out["f64"]["Nu"]
    for s in ("f32", "f16"):
        out[s]["abs_err_vs_f64"] = abs(out[s]["Nu"] - ref)
        out[s]["rel_err_vs_f64"] = abs(out[s]["Nu"] - ref) / abs(ref)
    state = (f"FP64 run until both residuals < {tol:g} (reached {reached[0]:.2e} / {reached[1]:.2e} "
             f"after {steps} steps)" if converged else
             f"FP64 run {steps} steps (cap {max_steps}); residuals there {reached[0]:.2e} / {reached[1]:.2e}, "
             f"above the {tol:g} target")
    return {
        "workload": f"cavity {n}x{n}, eps 0.6, Da 1e-2, Ra 1e5, Pr 1; {state}; "
                    "FP32/FP16 run the same number of steps",
        "converged": bool(converged), "residual_target": tol,
        "residual_reached": {"u": reached[0], "T": reached[1]}, "steps": steps,
        "results": out,
        "paper_context": {"Nu": 3.463, "grid": "120x120", "source": "Table Tab:Square1"},
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(n, budget_s, threads):
    """The FP64 oracle on the n x n throughput cavity, stepped until budget_s has passed,
    in a child process with `threads` OpenMP threads.  Returns (steps, seconds, threads)."""
    import subprocess
    code = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "import workloads as W\n"
        "from oracle import oracle as O\n"
        "o = O.Oracle(W.large_cavity(%d, storage='f64'))\n"
        "steps, t0 = 0, time.time()\n"
        "while True:\n"
        "    o.step(1); steps += 1; el = time.time() - t0\n"
        "    print('cpu baseline: step %%d, %%.1f s' %% (steps, el), file=sys.stderr, flush=True)\n"
        "    if el > %f: break\n"
        "print(json.dumps({'steps': steps, 's': el}))\n" % (ROOT, n, budget_s))
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    sys.stderr.write(r.stderr[-400:])
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    return rec["steps"], rec["s"], threads


def cpu_baseline(W, n, budget_s=15.0):
    """The FP64 oracle on the same workload (the n x n cavity) for a bounded number of
    steps: all host threads (OpenMP over rows), then one thread."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    st, el, _ = _oracle_steps(n, budget_s, threads)
    st1, el1, _ = _oracle_steps(n, budget_s, 1)
    return {"value": n * n * st / el / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} cavity, {st} full time steps after initialisation, FP64, "
                      f"OpenMP over rows ({threads} threads)",
            "single_thread": {"value": n * n * st1 / el1 / 1e6, "unit": "MLUPS", "cores": 1,
                              "sample": f"{n}x{n} cavity, {st1} full time steps, one thread"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--storage", default="f32", choices=("f32", "f16", "f64"))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--fusion", type=int, default=None, choices=(1, 2),
                    help="time steps per pass (default: the library's choice, 2 on large grids)")
    ap.add_argument("--ensemble-steps", type=int, default=10000)
    ap.add_argument("--no-ensemble-capped", action="store_true")
    ap.add_argument("--copy-reference-gib", type=float, default=0.0,
                    help="first run a plain device-to-device copy of this size, as the "
                         "reference for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path "
              "(domain decomposition with halo exchange) is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_1505_02976_amd import lbm

    if args.copy_reference_gib > 0:
        nbytes = int(args.copy_reference_gib * 2 ** 30)
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: reference copy of {nbytes} bytes done")
        del a, b

    n = args.size
    log(f"bench: {n}x{n} cavity, {args.storage}, warmup {args.warmup}, steps {args.steps}")
    main_res = timed_run(lbm, torch, W.large_cavity(n, storage=args.storage), args.warmup, args.steps,
                         fusion=args.fusion)
    log(f"bench: {main_res['mlups']:.0f} MLUPS, {main_res['main_kernel']} {main_res['main_GBps']:.0f} GB/s")

    modes = {}
    if not args.no_modes:
        for s in ("f16", "f64", "f32"):
            if s == args.storage:
                modes[s] = main_res
                continue
            k = max(100, args.steps // 5)
            modes[s] = timed_run(lbm, torch, W.large_cavity(n, storage=s), min(args.warmup, 100), k,
                                 fusion=args.fusion)
            log(f"bench: {s}: {modes[s]['mlups']:.0f} MLUPS, {modes[s]['main_kernel']} {modes[s]['main_GBps']:.0f} GB/s")

    one_step = None
    if not args.no_modes and main_res["steps_per_pass"] == 2:
        one_step = timed_run(lbm, torch, W.large_cavity(n, storage=args.storage), min(args.warmup, 100),
                             max(100, args.steps // 5), fusion=1)
        log(f"bench: {args.storage} one step per pass: {one_step['mlups']:.0f} MLUPS")

    ens = ens_c = None
    if not args.no_ensemble:
        ens = ensemble_run(lbm, torch, W, steps=args.ensemble_steps)
        log(f"bench: ensemble {ens['mlups']:.0f} MLUPS aggregate, {ens['nonfinite_problems']} non-finite")
        if not args.no_ensemble_capped:
            ens_c = ensemble_run(lbm, torch, W, steps=args.ensemble_steps, max_cell_re=5.0)
            log(f"bench: ensemble with Ra capped at cell Reynolds number 5: {ens_c['mlups']:.0f} MLUPS "
                f"aggregate, {ens_c['nonfinite_problems']} non-finite")
    adj = None
    if not args.no_adjoint:
        adj = adjoint_run(lbm, torch, W)
        log(f"bench: adjoint forward {adj['forward_s']:.2f} s, backward {adj['backward_s']:.2f} s "
            f"({adj['backward_us_per_step']:.0f} us per step)")
    td = None
    if not args.no_3d:
        td = three_d_run(torch, W)
        log(f"bench: 3-D f64 {td['f64']['mlups']:.0f} MLUPS ({td['f64']['GBps']:.0f} GB/s), "
            f"f32 {td['f32']['mlups']:.0f} MLUPS ({td['f32']['GBps']:.0f} GB/s), "
            f"f16 {td['f16']['mlups']:.0f} MLUPS ({td['f16']['GBps']:.0f} GB/s)")
    acc = None if args.no_accuracy else accuracy(lbm, W)
    cpu = None if args.no_cpu else cpu_baseline(W, n)

    line = {
        "metric": "MLUPS (flow+thermal) and % HBM roofline, FP32/FP16 vs FP64 at stated Nu error",
        "value": main_res["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"porous cavity {n}x{n}, eps 0.4, Da 1e-4, Ra 1e7, Pr 0.71, "
                               f"{args.storage} population storage",
                   "nodes": n * n, "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": main_res["main_GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": main_res["frac"],
                     "traffic": measured_traffic(main_res["main_kernel"], args.storage, n),
                     "kernel": main_res["main_kernel"],
                     "steps_per_launch": main_res["steps_per_pass"],
                     "bytes_per_launch": main_res["main_bytes_per_launch"],
                     "avg_launch_us": main_res["main_kernel_us"]},
        "modes": {s: {k: v for k, v in r.items()} for s, r in modes.items()},
        "one_step_per_pass": one_step,
        "ensemble": ens,
        "ensemble_capped": ens_c,
        "adjoint": adj,
        "three_d": td,
        "accuracy": acc,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
