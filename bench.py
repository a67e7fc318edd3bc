"""Benchmark of the characteristic (spatial-advection) step on one MI355X.

Default workload (the largest single-GPU configuration): 64^3 x-nodes on [-16,16)^3
times 32^3 k-nodes on [-4,4)^3 (8,589,934,592 phase-space points, 34 GB in FP32), one
GPU's share of the paper's 6-D grids; patches of 16 cells, ghost width 8, dt = 0.02,
seeded 8-packet Gaussian mixture, FP32 storage and arithmetic, FP64 mass and L2
recorded after every step.  A step is one pass of the whole hot path: the x1, x2 and
x3 sweeps of every point.  The x-cube does not fit in LDS, so the SLAB schedule runs:
a call of K steps alternates the sweep order between steps and takes K + 1 passes
over the field (one read and one write each), i.e. close to the method's 8 bytes per
point-update.

The field is resident in HBM before timing starts.  Before the W warmup steps the GPU
is brought to its steady state by about 0.4 s of the same kernels on a scratch copy
of the field (settle_steps).  The K timed steps are one library call (graph replays
back to back on the library's stream) between two HIP events; value, ms_per_step and
the roofline come from that interval.  A separate latency pass of L one-step calls,
with a HIP event recorded after each, gives the latency of an isolated step
(p50/p99).  Beside it: the plain FP64 form on the same grid (three launches per step,
eager) and the FP64 CPU oracle timed on a bounded sample of k-points (cpu_baseline),
whose result at those k-points also gives the error of the timed GPU run.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Other workloads (one JSON line each): --workload C2 (32^3 x 16^3, 134M points, the
x-cube in LDS: one launch per step; the 537 MB field is partly served by the 256 MB
memory-side cache), --workload C3 (48^3 x 24^3, autotuned patch / ghost / schedule),
--workload serving (200 Poisson-arriving requests of mixed grids under a 200 GB HBM
budget, continuous batching; p50/p99 step latency and aggregate point-updates/s),
--workload theta / lpc1 / ho2d (the next rows: Theta_V, the LPC1 step, the 2-D
harmonic oscillator).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["chasm_line.hpp", "chasm_kernels.hpp", "chasm_launch.hpp"]
THETA_FLOPS_FILE = os.path.join(ROOT, "profiles", "theta_flops.json")
THETA_SOURCES = ["chasm_theta.hip", "chasm_theta.hpp", "chasm_theta_big.hpp", "chasm_fft.hpp"]


def kernel_digest(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2205_02380_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, shape=None):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None when the
    kernel sources changed since the counters were taken, or when `shape` (N, patch,
    ghost) is given and the counted kernel was built for another one."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("kernel_digest") != kernel_digest():
        return None
    if shape is not None and "<float, %d, %d, %d," % tuple(shape) not in e.get("kernel", ""):
        return None
    return e.get("hbm_bytes_per_launch")


def step_traffic(sched: str, workload: str, shape=None, steps: int = 0):
    """Measured HBM bytes per step: the cube kernel; for the paired SLAB schedule the
    K + 1 passes of a K-step call (slab x2x1x1x2 and pencil x3x3 alternate) per step;
    None when no current counter run covers the kernels."""
    if sched == "cube":
        return measured_traffic("k_cube", workload, shape)
    if sched == "slab":
        a, b = measured_traffic("k_slab", workload, shape), measured_traffic("k_pencil", workload, shape)
        if a is None or b is None:
            return None
        return (a + b) / 2.0 * (steps + 1) / steps if steps else (a + b) / 2.0
    return None


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    """Measured device copy rate (read + write bytes / time) of a plain 1 GiB copy: the
    practical HBM ceiling of this machine, reported beside the published peak."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (a.elapsed_time(b) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def settle(torch, dev, seconds=0.4, nbytes=1 << 28):
    """Plain device copies for about `seconds`, so that the timed work starts at the
    GPU's steady clocks.  Returns the number of copies."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        n += 20
    del src, dst
    return n


def settle_advect(torch, dev, f, g, patch, ghost, dt, schedule, seconds=0.4, out_of_place=False, tile=0):
    """Run the same advection kernels on a scratch copy of the field for about `seconds`:
    an idle GPU, or one that ran other kernels, runs the first tens of milliseconds of
    this kernel a few percent slower.  The copy holds the field's own values (an all-zero
    field runs about 7 % faster) and shape, so every dispatch of these kernels in a
    profile of the run is alike.  The measured field is not touched.  Returns the steps
    run."""
    from paper_2205_02380_amd import chasm
    scratch = f.clone()
    adv = chasm.Advect(scratch, g, patch, ghost, dt, schedule=schedule, graph=True, out_of_place=out_of_place,
                       tile=tile)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        adv.step(8)
        torch.cuda.synchronize()
        n += 8
    adv.close()
    del scratch
    return n


def time_steps(adv, torch, steps, stream):
    """Exactly `steps` steps as one library call between two events: seconds."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    adv.step(steps)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3


def step_latencies(adv, torch, steps, stream):
    """Latency pass: one step per call with an event after each; per-step ms."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(steps):
        adv.step(1)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])


METRIC = "6-D point-updates/s FP32 vs FP64 plain at <=1e-5 rel err; p50/p99 step latency"


def oracle_sample(g, w, cubes, kidx, nst):
    """cpu_baseline leg: the FP64 oracle on a k-point sample, timed on the host cores."""
    import oracle
    nthreads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref = oracle.advect6d(cubes, g.nx, g.hx, g.nk, g.k_lo, g.hk, w.patch, w.ghost, w.dt, nst, kidx=kidx,
                          nthreads=nthreads)
    tc = time.perf_counter() - t0
    cpu = {"value": len(kidx) * g.cube * nst / tc, "unit": "point-updates/s", "cores": nthreads, "kind": "oracle",
           "sample": f"{len(kidx)} seeded k-points x {g.cube} x-points x {nst} steps "
                     f"({tc:.1f} s wall, FP64, OpenMP over k-points)"}
    return cpu, ref


def bench_large(args, name):
    """C3 / C4: one large FP32 job, graph-replayed steps, per-step FP64 diagnostics."""
    import dataclasses

    import torch
    from paper_2205_02380_amd import autotune, chasm, inputs
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    w = inputs.workload(name)
    copy_gbs = copy_bandwidth(torch, dev)
    tuning = None
    if name == "C3" and not args.no_tune:
        # timed as the run below: graph-replayed, FP64 diagnostics every step
        res = autotune.tune(w.grid, w.dt, w.packets, steps=5, tol=1e-5, reduce_each_step=True,
                            log=lambda m: print(m, file=sys.stderr, flush=True))
        b = res["best"]
        tuning = {"best": b, "candidates": len(res["candidates"]),
                  "table_columns": ["patch", "ghost", "schedule", "tile", "out_of_place", "ms_per_step", "deviation"],
                  "table": [[c["patch"], c["ghost"], c["schedule"], c["tile"], c["out_of_place"],
                             round(c["ms_per_step"], 3), float("%.3g" % c["deviation"])] for c in res["candidates"]]}
        w = dataclasses.replace(w, patch=(b["patch"],) * 3, ghost=b["ghost"])
        sched = b["schedule"]
        oop = b["out_of_place"]
        tile = b["tile"]
    else:
        sched = "auto"
        oop = False                 # measured on C4: in place 26.8 ms per step, out of place 27.5
        tile = 0
    g = w.grid
    f = torch.empty(g.shape(), dtype=torch.float32, device=dev)
    coef, gx, gk = inputs.packet_factors(g, w.packets)
    inputs.fill_separable(f, coef, gx, gk)
    # the oracle sample is bounded to about 20 s of host work: 96 k-points of C4 (64^3
    # cubes, 160 steps) took 66 s on 16 cores, so C4 samples 32; C3's 96 take about 7 s
    kidx = inputs.k_sample(g, (args.cpu_kpoints or (32 if name == "C4" else 96)) / g.nkpts, 40)
    start = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    steps = args.steps
    lat = min(steps, args.latency_steps)
    nall = args.warmup + steps + lat
    adv = chasm.Advect(f, g, w.patch, w.ghost, w.dt, schedule=sched, graph=True, reduce_each_step=True,
                       history_cap=nall, stream=stream, out_of_place=oop, tile=tile)
    sched = adv.schedule
    settled = settle_advect(torch, dev, f, g, w.patch, w.ghost, w.dt, sched, out_of_place=oop, tile=tile)
    adv.step(args.warmup)
    total_s = time_steps(adv, torch, steps, stream)
    per = step_latencies(adv, torch, lat, stream)
    hist = adv.history(nall)
    adv.close()
    got = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    del f
    torch.cuda.empty_cache()
    value = g.points * steps / total_s
    # the method's bytes: one FP32 read and one write of every point per step
    achieved = 8.0 * g.points / (total_s / steps) / 1e9
    sched_bpp = 8.0 if sched == "cube" else (8.0 * (steps + 1) / steps if sched == "slab" else 24.0)

    # ---- plain FP64 one-job form on the same grid ---------------------------------
    fp64 = None
    if not args.no_fp64:
        f64 = torch.empty(g.shape(), dtype=torch.float64, device=dev)
        inputs.fill_separable(f64, *inputs.packet_factors(g, w.packets))
        adv64 = chasm.Advect(f64, g, w.patch, w.ghost, w.dt, schedule="plain", stream=stream)
        adv64.step(1)
        n64 = max(2, min(args.fp64_steps, 10))
        t64 = time_steps(adv64, torch, n64, stream)
        adv64.close()
        del f64
        torch.cuda.empty_cache()
        fp64 = {"value": g.points * n64 / t64, "unit": "point-updates/s", "ms_per_step": t64 * 1e3 / n64,
                "steps": n64, "schedule": "plain (3 launches/step, eager)", "alg_bytes_per_point_update": 48}

    cpu = err = None
    if not args.no_cpu:
        nst = min(nall, args.cpu_steps) if args.cpu_steps else nall
        cpu, ref = oracle_sample(g, w, start, kidx, nst)
        if nst == nall:
            err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    m0 = hist[0, 0, 0]
    kern = {"cube": "k_cube", "slab": "k_slab (x2 x1 | x1 x2) and k_pencil (x3 | x3), alternating",
            "plain": "k_slab (x1), k_pencil (x2), k_pencil (x3)"}[sched]
    return {
        "metric": METRIC, "value": value, "unit": "point-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": total_s * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded Gaussian-packet mixture, generated on the GPU)",
        "config": {"workload": f"{w.name}: {g.nx[0]}^3 x [{g.x_lo[0]:g},{g.x_hi[0]:g})^3 by {g.nk[0]}^3 k "
                               f"[{g.k_lo[0]:g},{g.k_hi[0]:g})^3, {g.points} points, patch {w.patch[0]}, "
                               f"ghost {w.ghost}, dt {w.dt}, FP32, one job, FP64 mass/L2 every step",
                   "schedule": sched, "graph": True, "out_of_place": oop},
        "step_latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                            "mean": float(per.mean()), "steps": lat,
                            "pass": "separate, after the timed steps: one-step calls, an event after each"},
        "settle_steps": settled, "steps_total": nall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": step_traffic(sched, name, (g.nx[0], w.patch[0], w.ghost), steps),
                     "kernel": "whole step: " + kern, "alg_bytes_per_point_update": 8.0,
                     "schedule_bytes_per_point_update": sched_bpp, "measured_copy_GBs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs},
        "fp64_plain": fp64, "fp32_vs_fp64_plain": None if fp64 is None else value / fp64["value"],
        "mass_drift": float(abs(hist[-1, 0, 0] - m0) / abs(m0)), "l2_last": float(hist[-1, 0, 1]),
        "autotune": tuning, "err_vs_oracle": err, "cpu_baseline": cpu,
    }


def bench_serving(args):
    import torch
    from paper_2205_02380_amd import inputs, serve
    trace = inputs.serving_trace()
    be = serve.ChasmBackend()
    # warm the kernels of every shape class once
    warm = [inputs.Request(-1 - i, 0.0, gr, 1, 0.02, inputs.random_packets(1, 1)) for i, gr in
            enumerate(inputs.SERVING_SHAPES)]
    serve.Server(be, budget_bytes=200e9, max_active=64).run(warm)
    torch.cuda.synchronize()
    rep = serve.Server(be, budget_bytes=200e9, max_active=64).run(trace)
    d = rep.as_dict()
    return {
        "metric": METRIC, "value": rep.throughput, "unit": "point-updates/s", "n_gpus": 1, "steps": rep.ticks,
        "warmup": len(warm), "ms_per_step": rep.makespan_s * 1e3 / max(rep.ticks, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded request trace and Gaussian-packet fields)",
        "config": {"workload": "serving: 200 requests, Poisson 20/s, grids {16^3x8^3, 24^3x12^3, 32^3x16^3, "
                               "48^3x16^3}, steps U[10,200], dt {0.01,0.02,0.05}, 200 GB HBM budget, "
                               "continuous batching", "patch": 8, "ghost": 6},
        "step_latency_ms": {"p50": d["p50_step_ms"], "p99": d["p99_step_ms"]},
        "serving": d, "roofline": None, "cpu_baseline": None,
    }


THETA_FLOP_NOTE = ("conventional count of one period-2N_k FFT convolution per x-point and nucleus: "
                   "2 x 5 P^3 log2(P^3) + 2 P^3 flops, P = 2 N_k")
THETA_EXECUTED_NOTE = ("executed FP64 flops per x-point and nucleus: 64 lanes x (ADD + MUL + TRANS + 2 FMA) "
                       "FP64 wave instructions of the Theta_V kernels, from rocprofv3 counters "
                       "(profiles/theta_flops.json)")


def theta_executed_flops_per_xpoint(nk: int):
    """FP64 flops the Theta_V kernels execute per x-point (one nucleus), from the
    committed rocprofv3 counter runs, or None when the Theta_V sources changed since."""
    try:
        with open(THETA_FLOPS_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(str(nk))
    if not e or e.get("kernel_digest") != kernel_digest(THETA_SOURCES):
        return None
    return e.get("executed_flops_per_xpoint")


def theta_roofline(nk: int, xpoints: int, applies: int, seconds: float, kernel: str) -> dict:
    """Roofline of `applies` Theta_V evaluations per x-point in `seconds`, priced on the
    executed FP64 flops when the counters match the sources (else on the conventional
    FFT count), against the FP64 vector peak; the conventional figure rides along."""
    conv = theta_flops_per_xpoint(nk) * xpoints * applies / seconds / 1e12
    ex = theta_executed_flops_per_xpoint(nk)
    r = {"bound": "alu", "peak": 78.6, "unit": "TFLOP/s", "traffic": None, "kernel": kernel,
         "conventional": {"achieved": conv, "frac": conv / 78.6, "flop_count": THETA_FLOP_NOTE}}
    if ex is None:
        r.update(achieved=conv, frac=conv / 78.6, flop_count=THETA_FLOP_NOTE + " (executed count unavailable: "
                 "the Theta_V sources changed since the counters were taken)")
    else:
        a = ex * xpoints * applies / seconds / 1e12
        r.update(achieved=a, frac=a / 78.6, flop_count=THETA_EXECUTED_NOTE,
                 executed_flops_per_xpoint=ex)
    return r


def theta_flops_per_xpoint(nk: int) -> float:
    P3 = (2 * nk) ** 3
    return 2 * 5 * P3 * np.log2(P3) + 2 * P3


def bench_theta(args):
    """Theta_V^T (Sec. 4) on the paper's x-grid of Sec. 5.2: 61^3 x-nodes on [-9, 9]^3 by
    N_k^3 k-nodes on [-6.4, 6.4)^3 (N_k = 16: dk = 0.8, the paper's grid; N_k = 32 refines
    dk on the same k-box and runs the staged transforms), one nucleus at the
    origin, FP32 field, FP64 arithmetic."""
    import torch
    from paper_2205_02380_amd import inputs, theta
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    nk = args.nk
    grid = inputs.Grid((61,) * 3, (-9.0,) * 3, (9.3,) * 3, (nk,) * 3, (-6.4,) * 3, (6.4,) * 3)
    pk = inputs.random_packets(4, 21, c_range=(-3.0, 3.0), k0_range=(-1.0, 1.0), s_range=(0.8, 1.5))
    f = torch.empty(grid.shape(), dtype=torch.float32, device=dev)
    coef, gx, gk = inputs.packet_factors(grid, pk)
    inputs.fill_separable(f, coef, gx, gk)
    out = torch.empty_like(f)
    th = theta.Theta(grid, [(0.0, 0.0, 0.0)], dtype="f32", stream=stream)
    settle(torch, dev)
    for _ in range(args.warmup):
        th.apply(f, out)
    torch.cuda.synchronize()
    steps = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        th.apply(f, out)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    total_s = ev[0].elapsed_time(ev[steps]) / 1e3
    npts = grid.cube
    mean_s = float(per.mean()) / 1e3
    cpu = None
    if not args.no_cpu:
        from oracle import tkm
        rng = np.random.default_rng(23)
        xidx = np.stack([rng.integers(0, 61, {16: 16, 32: 4}[nk]) for _ in range(3)], axis=1)
        fx = [f[:, :, :, i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in xidx]
        t0 = time.perf_counter()
        for n, (i1, i2, i3) in enumerate(xidx):
            tkm.theta_point(fx[n], (grid.x_axis(0)[i1], grid.x_axis(1)[i2], grid.x_axis(2)[i3]), grid.k_lo, grid.hk)
        tc = time.perf_counter() - t0
        cpu = {"value": len(xidx) * grid.nkpts / tc, "unit": "point-evaluations/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(xidx)} seeded x-points x {grid.nkpts} k-points ({tc:.1f} s, numpy FP64, threefold "
                         "transforms)"}
    th.close()
    kern = "whole apply (transpose, k_theta, transpose)" if nk <= 16 else "whole apply (k_thA, k_thBCD, k_thE)"
    return {
        "metric": "Theta_V^T point-evaluations/s (truncated kernel method, FP64 arithmetic)",
        "value": grid.points * steps / total_s, "unit": "point-evaluations/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": total_s * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (f32 field)", "data": "synthetic (seeded Gaussian-packet mixture)",
        "config": {"workload": f"theta: 61^3 x [-9,9]^3 by {nk}^3 k [-6.4,6.4)^3, {grid.points:,} points, one "
                               "nucleus, FP32 field, FP64 transforms"},
        "step_latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                            "mean": float(per.mean())},
        "roofline": theta_roofline(nk, npts, 1, mean_s, kern),
        "cpu_baseline": cpu,
    }


def bench_lpc1(args):
    """Full LPC1 steps of the Wigner-Coulomb equation (Sec. 2.2): the characteristic step
    and two truncated-kernel Theta_V evaluations per step.  Hydrogen (one proton at the
    origin) on the paper's x-grid of Sec. 5.2: 61^3 nodes on [-9, 9]^3 (dx = 0.3, four
    patches of 15 cells per axis, n_nb = 15; this line has no compiled kernels, so the
    characteristic step runs on the runtime-shape kernels), by N_k^3 k-nodes on
    [-6.4, 6.4)^3 (N_k = 16: dk = 0.8; N_k = 32: dk = 0.4, staged Theta_V), tau = 0.025,
    FP32 field."""
    import torch
    from paper_2205_02380_amd import inputs, lpc1
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    nk = args.nk
    grid = inputs.Grid((61,) * 3, (-9.0,) * 3, (9.3,) * 3, (nk,) * 3, (-6.4,) * 3, (6.4,) * 3)
    pk = inputs.random_packets(4, 31, c_range=(-3.0, 3.0), k0_range=(-1.0, 1.0), s_range=(0.8, 1.5))
    f = torch.empty(grid.shape(), dtype=torch.float32, device=dev)
    coef, gx, gk = inputs.packet_factors(grid, pk)
    inputs.fill_separable(f, coef, gx, gk)
    tau = 0.025
    s = lpc1.LPC1(f, grid, 15, 15, tau, [(0.0, 0.0, 0.0)], stream=stream)
    settle(torch, dev)
    s.step(args.warmup)
    torch.cuda.synchronize()
    steps = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        s.step(1)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    s.close()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    total_s = ev[0].elapsed_time(ev[steps]) / 1e3
    cpu = None
    if not args.no_cpu:
        from oracle import lpc1 as olpc1
        sx = 8 if nk == 16 else 4
        small = inputs.Grid((sx,) * 3, (-0.15 * sx,) * 3, (0.15 * sx,) * 3, (nk,) * 3, (-6.4,) * 3, (6.4,) * 3)
        f0 = inputs.gaussian_field(small, pk).numpy()
        t0 = time.perf_counter()
        olpc1.lpc1(f0, small, sx // 2, sx // 2 - 1, tau, 1, [(0.0, 0.0, 0.0)], [1.0], direct=False)
        tc = time.perf_counter() - t0
        cpu = {"value": small.points / tc, "unit": "point-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"one LPC1 step of a {sx}^3 x {nk}^3 grid ({small.points} points, {tc:.1f} s; numpy/C FP64)"}
    return {
        "metric": "LPC1 point-updates/s (Wigner-Coulomb step: advection + 2 truncated-kernel Theta_V)",
        "value": grid.points * steps / total_s, "unit": "point-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": total_s * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 field, f64 Theta", "data": "synthetic (seeded Gaussian-packet mixture)",
        "config": {"workload": f"lpc1: 61^3 x [-9,9]^3 (dx 0.3) by {nk}^3 k [-6.4,6.4)^3, {grid.points:,} points, "
                               "one proton, 4 patches of 15 cells, n_nb 15, tau 0.025"},
        "step_latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                            "mean": float(per.mean())},
        "roofline": theta_roofline(nk, grid.cube, 2, float(per.mean()) / 1e3,
                                   "whole step (two Theta evaluations dominate)"),
        "cpu_baseline": cpu,
    }


def bench_ho2d(args):
    """The 2-D harmonic oscillator of Sec. 5.1 on the paper's grid and time step: x on
    [-12, 12] with dx = 0.1 (241 nodes, 4 patches, n_nb = 20), k on [-6.4, 6.4) with
    dk = 0.025 (512 nodes), omega = (pi/5)^2, tau = 2e-5, zero inflow, one full period
    T = 10 (500000 LPC1 steps), against the exact phase-space rotation."""
    import math

    import torch
    from oracle import ho2d as oho
    from paper_2205_02380_amd import ho2d
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    W = (math.pi / 5.0) ** 2
    nx, hx, nk, hk, tau = 241, 0.1, 512, 0.025, 0.00002
    steps = args.steps if args.steps != 100 else 500000
    x, k = oho.axes(nx, -12.0, hx, nk, -6.4, hk)
    f0 = oho.f0(x[None, :], k[:, None])
    f = torch.tensor(f0, dtype=torch.float64, device=dev)
    s = ho2d.HO2D(f, nx, -12.0, hx, nk, -6.4, hk, 60, 20, W, tau, stream=stream)
    g = torch.tensor(f0, dtype=torch.float64, device=dev)
    w = ho2d.HO2D(g, nx, -12.0, hx, nk, -6.4, hk, 60, 20, W, tau, stream=stream)
    w.step(args.warmup)
    w.close()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    s.close()
    total_s = e0.elapsed_time(e1) / 1e3
    got = f.cpu().numpy()
    ex = oho.exact(x, k, steps * tau, W)
    err_inf = float(np.max(np.abs(got - ex)))
    err_2 = float(np.sqrt(np.sum((got - ex) ** 2) * hx * hk))
    mass_dev = float(abs(got.sum() - f0.sum()) * hx * hk)
    cpu = None
    if not args.no_cpu:
        n = 10
        t0 = time.perf_counter()
        oho.lpc1(f0, x, k, hx, hk, 60, 20, W, tau, n)
        tc = time.perf_counter() - t0
        cpu = {"value": nx * nk * n / tc, "unit": "point-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"{n} LPC1 steps of the same grid ({tc:.1f} s; C line oracle + numpy FFT, FP64)"}
    pts = nx * nk
    # Conventional FP64 flops of one step: two k-derivatives by transforms (a forward and
    # an inverse complex transform of nk points, 5 nk log2 nk flops each, and the 6 nk of
    # the multiply, per pair of x columns) and the x-advection of 2 nk lines (interface
    # slopes, the patch solves as products with the patch inverses, the 4-tap evaluation).
    P, M, g = 4, 60, 20
    ncl = (nx + 1) // 2
    dk = ncl * (2 * 5 * nk * math.log2(nk) + 6 * nk)
    adv_line = 2 * (P + 1) * (2 * g + 1) + 2 * (M + 1) ** 2 * P + 2 * 4 * nx
    flops = (2 * dk + 2 * nk * adv_line) * steps
    return {
        "metric": "2-D harmonic-oscillator LPC1 point-updates/s (FP64) and eps_inf(T=10) vs the exact rotation",
        "value": pts * steps / total_s, "unit": "point-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": total_s * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "analytic initial packet of Sec. 5.1",
        "config": {"workload": "ho2d: x 241 nodes dx 0.1 on [-12,12], k 512 nodes dk 0.025 on [-6.4,6.4), "
                               "4 patches, n_nb 20, omega (pi/5)^2, tau 2e-5, zero inflow, T = steps x tau"},
        "accuracy": {"eps_inf": err_inf, "eps_2": err_2, "mass_deviation": mass_dev, "t": steps * tau},
        "roofline": {"bound": "alu", "achieved": flops / total_s / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": flops / total_s / 1e12 / 78.6, "traffic": None,
                     "kernel": "whole step (k_ho_dk512 twice on 121 one-wave blocks, k_ho_advect once on 512 blocks); "
                               "the 1 MB working set stays in cache and each launch is a short dependent chain, so "
                               "the step is bound by latency, far from either roofline",
                     "flop_count": "per step: 2 x (nx+1)/2 x (10 nk log2 nk + 6 nk) for the derivatives plus "
                                   "2 nk x (2 (P+1)(2g+1) + 2 (M+1)^2 P + 8 nx) for the advection"},
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--cpu-kpoints", type=int, default=0,
                    help="k-points of the oracle sample (default: 24 for C2, 96 for C3, 32 for C4)")
    ap.add_argument("--latency-steps", type=int, default=50,
                    help="steps of the separate per-step latency pass (at most --steps)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--workload", default="C4", choices=["C2", "C3", "C4", "serving", "theta", "lpc1", "ho2d"])
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--nk", type=int, default=16, choices=[16, 32],
                    help="k-nodes per axis of the theta and lpc1 workloads (61^3 x 64^3 FP32 is 238 GB a field)")
    ap.add_argument("--cpu-steps", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain device copy of 1 GiB (the reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: --gpus {args.gpus} is not supported "
              "(the advection is independent per k-point; see the sharding notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2205_02380_amd import chasm, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.calibrate_copy:
        # 2^28 floats read and 2^28 floats written: 1 GiB each way
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload in ("C3", "C4"):
        print(json.dumps(bench_large(args, args.workload)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(bench_serving(args)), flush=True)
        return
    if args.workload == "theta":
        print(json.dumps(bench_theta(args)), flush=True)
        return
    if args.workload == "lpc1":
        print(json.dumps(bench_lpc1(args)), flush=True)
        return
    if args.workload == "ho2d":
        print(json.dumps(bench_ho2d(args)), flush=True)
        return
    w = inputs.workload("C2")
    g = w.grid
    points = g.points
    copy_gbs = copy_bandwidth(torch, dev)

    # ---- FP32, cube schedule, graph replay ------------------------------------------
    f = torch.empty(g.shape(), dtype=torch.float32, device=dev)
    coef, gx, gk = inputs.packet_factors(g, w.packets)
    inputs.fill_separable(f, coef, gx, gk)
    kidx = inputs.k_sample(g, (args.cpu_kpoints or 24) / g.nkpts, 40)
    start_cubes = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    torch.cuda.synchronize()
    adv = chasm.Advect(f, g, w.patch, w.ghost, w.dt, graph=True, stream=stream)
    sched = adv.schedule
    lat = min(args.steps, args.latency_steps)
    nall = args.warmup + args.steps + lat
    settled = settle_advect(torch, dev, f, g, w.patch, w.ghost, w.dt, sched)
    adv.step(args.warmup)
    total_s = time_steps(adv, torch, args.steps, stream)
    per = step_latencies(adv, torch, lat, stream)
    adv.close()
    value = points * args.steps / total_s
    ms_per_step = total_s * 1e3 / args.steps
    kernel = "k_cube" if sched == "cube" else "k_slab+k_pencil"
    bytes_alg = 8.0 * points                       # read + write of every FP32 value, once per launch
    mean_kernel_s = total_s / args.steps           # one launch per step, back to back
    achieved = bytes_alg / mean_kernel_s / 1e9
    gpu_cubes = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    del f
    torch.cuda.empty_cache()

    # ---- plain FP64 one-job form ---------------------------------------------------------
    value64 = t64 = None
    if not args.no_fp64:
        f64 = torch.empty(g.shape(), dtype=torch.float64, device=dev)
        inputs.fill_separable(f64, coef, gx, gk)
        adv64 = chasm.Advect(f64, g, w.patch, w.ghost, w.dt, schedule="plain", stream=stream)
        adv64.step(2)
        t64 = time_steps(adv64, torch, args.fp64_steps, stream)
        adv64.close()
        value64 = points * args.fp64_steps / t64
        del f64
        torch.cuda.empty_cache()

    # ---- CPU baseline: the FP64 oracle on a bounded k-sample ---------------------------
    cpu = None
    err = None
    if not args.no_cpu:
        cpu, ref = oracle_sample(g, w, start_cubes, kidx, nall)
        err = float(np.max(np.abs(gpu_cubes - ref)) / np.max(np.abs(ref)))

    traffic = measured_traffic(kernel, "C2", (g.nx[0], w.patch[0], w.ghost))
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 4-packet Gaussian mixture, generated on the GPU)",
        "config": {"workload": "32^3 x [-12,12)^3 by 16^3 k [-4,4)^3, 134217728 points, patch 8, ghost 6, "
                               "dt 0.02, FP32, one job", "schedule": sched, "graph": True},
        "step_latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                            "mean": float(per.mean()), "steps": lat,
                            "pass": "separate, after the timed steps, one event per step"},
        "settle_steps": settled, "steps_total": nall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                     "alg_bytes_per_launch": bytes_alg, "measured_copy_GBs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs},
        "fp64_plain": None if value64 is None else {
            "value": value64, "unit": "point-updates/s", "ms_per_step": t64 * 1e3 / args.fp64_steps,
            "schedule": "plain (3 launches/step, eager)", "alg_bytes_per_point_update": 48},
        "fp32_vs_fp64_plain": None if value64 is None else value / value64,
        "err_vs_oracle": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
