"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative to max|f|): FP64 <= 1e-12 per step (same algorithm, different
operation order: reduced Thomas vs dense pivoted LU, tabulated weights vs direct
B-spline sums); FP32 <= 1e-5 per step and <= 1e-4 after 100 steps (the bound the
workload specifies; a single FP32 sweep of smooth data is ~1e-7).  The oracle starts
from the same FP32-rounded initial field, widened to FP64, so only the sweep
arithmetic is compared.  Large grids compare sampled k-points with the oracle and
every point with the separable reference (the tensor product of oracle line sweeps).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2205_02380_amd import chasm, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def gpu_run(f_host, grid, patch, ghost, dt, steps, dtype, **kw):
    f = torch.tensor(np.ascontiguousarray(f_host), dtype=dtype, device=DEV)
    with chasm.Advect(f, grid, patch, ghost, dt, **kw) as a:
        a.step(steps)
        torch.cuda.synchronize()
    return f.double().cpu().numpy()


def oracle_full(f, grid, patch, ghost, dt, steps, closure=oracle.PMBC):
    P = (patch,) * 3 if isinstance(patch, int) else patch
    return oracle.advect6d(f, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, P, ghost, dt, steps, closure=closure)


# --------------------------------------------------------------------------- C1 (FP64)
_C1 = {}


def c1_reference(steps):
    w = inputs.workload("C1")
    if "f0" not in _C1:
        _C1["f0"] = inputs.gaussian_field(w.grid, w.packets).numpy()
    if steps not in _C1:
        _C1[steps] = oracle_full(_C1["f0"], w.grid, w.patch, w.ghost, w.dt, steps)
    return w, _C1["f0"], _C1[steps]


@pytest.mark.parametrize("schedule", ["cube", "slab", "plain"])
@pytest.mark.parametrize("steps,tol", [(1, 1e-12), (10, 1e-11)])
def test_c1_fp64_matches_oracle(schedule, steps, tol):
    w, f0, ref = c1_reference(steps)
    say(f"C1 fp64 schedule={schedule} steps={steps}")
    got = gpu_run(f0, w.grid, w.patch, w.ghost, w.dt, steps, torch.float64, schedule=schedule)
    assert rel(got, ref) < tol


@pytest.mark.parametrize("schedule", ["cube", "slab"])
def test_c1_poly3_carries_cubics_exactly(schedule):
    w = inputs.workload("C1")
    g = w.grid
    coeffs = inputs.cubic_coeffs(1)
    X = [g.x_axis(d) for d in range(3)]
    K = [g.k_axis(d) for d in range(3)]
    k3, k2, k1, x3, x2, x1 = np.meshgrid(K[2], K[1], K[0], X[2], X[1], X[0], indexing="ij", sparse=True)
    f0 = np.broadcast_to(inputs.cubic_eval(coeffs, x1, x2, x3), g.shape()).copy()
    steps = 10
    T = w.dt * steps
    exact = np.broadcast_to(inputs.cubic_eval(coeffs, x1 - k1 * T, x2 - k2 * T, x3 - k3 * T), g.shape())
    say(f"C1 poly3 cubic schedule={schedule}")
    got = gpu_run(f0, g, w.patch, w.ghost, w.dt, steps, torch.float64, schedule=schedule, closure="poly3")
    assert rel(got, exact) < 1e-11


# --------------------------------------------------------------------------- small shapes
SMALL = [
    # N, M, ghost, nk, dt*hk/h multiplier -> alpha steps
    (8, 2, 1, (3, 4, 5), 0.75),
    (8, 4, 3, (4, 3, 2), 1.0),      # integer shifts (alpha in Z)
    (8, 8, 7, (5, 2, 3), 0.4),
    (16, 4, 8, (4, 5, 3), 0.3),
    (16, 8, 15, (3, 3, 4), 1.25),   # untruncated stencils: the global spline
    (16, 16, 5, (2, 3, 4), 0.2),
    (24, 12, 6, (3, 4, 2), 0.55),
    (32, 16, 8, (2, 3, 4), 0.35),
]


@pytest.mark.parametrize("N,M,g,nk,amul", SMALL)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_small_shapes_every_schedule(N, M, g, nk, amul, dtype):
    """Ragged k grids, shifts of both signs, zero, integer and |alpha| >= 1, and
    every schedule the shape supports."""
    h = 0.5
    hk = 0.5
    grid = inputs.Grid((N, N, N), (-N * h / 2,) * 3, (N * h / 2,) * 3, nk,
                       tuple(-hk * (n // 2) for n in nk), tuple(hk * (n - n // 2) for n in nk))
    dt = amul * h / hk                      # alpha = k dt / h = amul * (k / hk)
    pk = inputs.random_packets(2, N + M, c_range=(-1.0, 1.0), s_range=(0.6, 1.0))
    f0 = inputs.gaussian_field(grid, pk).numpy()
    steps = 2
    tdtype = torch.float64 if dtype == "f64" else torch.float32
    start = f0 if dtype == "f64" else f0.astype(np.float32).astype(np.float64)
    ref = oracle_full(start, grid, M, g, dt, steps)
    tol = 1e-12 if dtype == "f64" else 1e-5
    scheds = ["cube", "slab", "plain"] if (dtype == "f32" or N <= 24) else ["slab", "plain"]
    for sched in scheds:
        say(f"small N={N} M={M} g={g} nk={nk} {dtype} {sched}")
        got = gpu_run(start, grid, M, g, dt, steps, tdtype, schedule=sched)
        assert rel(got, ref) < tol, sched


# --------------------------------------------------------------------------- C2 (FP32)
_C2 = {}


def c2_setup():
    if not _C2:
        w = inputs.workload("C2")
        f32 = inputs.gaussian_field(w.grid, w.packets, dtype=torch.float32)
        _C2.update(w=w, f32=f32, kidx=inputs.k_sample(w.grid, 0.004, 40))
    return _C2["w"], _C2["f32"], _C2["kidx"]


def c2_oracle_cubes(steps):
    w, f32, kidx = c2_setup()
    key = ("cubes", steps)
    if key not in _C2:
        start = np.stack([f32[i3, i2, i1].double().numpy() for i1, i2, i3 in kidx])
        _C2[key] = oracle.advect6d(start, w.grid.nx, w.grid.hx, w.grid.nk, w.grid.k_lo, w.grid.hk, w.patch, w.ghost,
                                   w.dt, steps, kidx=kidx)
    return _C2[key]


def test_c2_fp32_one_step():
    w, f32, kidx = c2_setup()
    ref = c2_oracle_cubes(1)
    say("C2 fp32 1 step")
    f = f32.to(DEV)
    with chasm.Advect(f, w.grid, w.patch, w.ghost, w.dt) as a:
        assert a.schedule == "cube"
        a.step(1)
    torch.cuda.synchronize()
    got = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    assert rel(got, ref) < 1e-5


def test_c2_fp32_100_steps_graph():
    """The benchmark's launch configuration: cube schedule, HIP graph, 100 steps."""
    w, f32, kidx = c2_setup()
    ref = c2_oracle_cubes(100)
    say("C2 fp32 100 steps graph")
    f = f32.to(DEV)
    with chasm.Advect(f, w.grid, w.patch, w.ghost, w.dt, graph=True) as a:
        a.step(100)
    torch.cuda.synchronize()
    got = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    err = rel(got, ref)
    say(f"  sampled k-points: {len(kidx)}, rel err {err:.3e}")
    assert err < 1e-4
    # every point against the separable reference (tensor product of oracle line sweeps)
    coef, U = oracle.separable_factors(w.grid, w.packets, w.patch, w.ghost, w.dt, 100)
    sep = torch.empty(w.grid.shape(), dtype=torch.float32, device=DEV)
    inputs.fill_separable(sep, coef, U)
    full_err = float((f - sep).abs().max() / sep.abs().max())
    say(f"  all points vs separable reference: {full_err:.3e}")
    assert full_err < 1e-4


def test_c2_schedules_agree():
    w, f32, _ = c2_setup()
    outs = {}
    for sched in ("cube", "slab", "plain"):
        f = f32.to(DEV)
        with chasm.Advect(f, w.grid, w.patch, w.ghost, w.dt, schedule=sched) as a:
            a.step(3)
        torch.cuda.synchronize()
        outs[sched] = f
    scale = float(outs["cube"].abs().max())
    for sched in ("slab", "plain"):
        d = float((outs[sched] - outs["cube"]).abs().max()) / scale
        say(f"C2 {sched} vs cube: {d:.3e}")
        assert d < 1e-6


def test_c2_reductions_match_oracle_on_stored_field():
    w, f32, _ = c2_setup()
    g = w.grid
    f = f32.to(DEV)
    with chasm.Advect(f, g, w.patch, w.ghost, w.dt) as a:
        a.step(5)
        m, l2, mom = a.mass()
    stored = f.double().cpu().numpy()
    ref = oracle.reduce(stored, g.nx, g.x_lo, g.hx, g.nk, g.k_lo, g.hk)
    assert m == pytest.approx(ref[0], rel=1e-12)
    assert l2 == pytest.approx(ref[1], rel=1e-12)
    for i in range(6):
        assert mom[i] == pytest.approx(ref[2 + i], rel=1e-10, abs=1e-12 * abs(ref[0]) * 16)


@pytest.mark.parametrize("graph", [False, True])
def test_reduce_each_step_history(graph):
    w = inputs.workload("C1")
    g = w.grid
    f0 = inputs.gaussian_field(g, w.packets).numpy().astype(np.float32)
    f = torch.tensor(f0, device=DEV)
    expect = []
    with chasm.Advect(f, g, w.patch, w.ghost, w.dt, reduce_each_step=True, graph=graph) as a:
        for s in range(6):
            a.step(1)
            torch.cuda.synchronize()
            st = f.double().cpu().numpy()
            expect.append(oracle.reduce(st, g.nx, g.x_lo, g.hx, g.nk, g.k_lo, g.hk))
        hist = a.history()
    assert hist.shape == (6, 1, 8)
    for s in range(6):
        for i in range(8):
            assert hist[s, 0, i] == pytest.approx(expect[s][i], rel=1e-12, abs=1e-14)


def test_graph_replay_equals_eager_bitwise():
    w = inputs.workload("C1")
    f0 = inputs.gaussian_field(w.grid, w.packets, dtype=torch.float32)
    a_out, b_out = f0.to(DEV), f0.to(DEV)
    with chasm.Advect(a_out, w.grid, w.patch, w.ghost, w.dt) as a:
        a.step(27)
    with chasm.Advect(b_out, w.grid, w.patch, w.ghost, w.dt, graph=True) as b:
        b.step(3)
        torch.cuda.synchronize()
        b.step(4)
        b.step(20)                  # two 8-step graphs and four single-step graphs
    torch.cuda.synchronize()
    assert torch.equal(a_out, b_out)


def test_batch_equals_single_runs_bitwise():
    w = inputs.workload("C1")
    fields = [inputs.gaussian_field(w.grid, inputs.random_packets(2, 50 + i), dtype=torch.float32) for i in range(3)]
    batch = torch.stack(fields).to(DEV).contiguous()
    with chasm.Advect(batch, w.grid, w.patch, w.ghost, w.dt, reduce_each_step=True) as a:
        a.step(4)
        diag = a.diagnostics()
    torch.cuda.synchronize()
    for i, f0 in enumerate(fields):
        f = f0.to(DEV)
        with chasm.Advect(f, w.grid, w.patch, w.ghost, w.dt) as s:
            s.step(4)
            d1 = s.diagnostics()
        torch.cuda.synchronize()
        assert torch.equal(f, batch[i])
        assert np.allclose(diag[i], d1[0], rtol=1e-13, atol=0)


def test_step_many_equals_individual_runs():
    """Handles with the same kernels share one launch per sweep (a work list of jobs with
    their own fields, dt and k grids); each result equals the job run alone, bitwise."""
    jobs = []
    specs = [(16, 8, 2.0, 0.01, 5), (16, 8, 2.0, 0.05, 7), (24, 12, 3.0, 0.02, 9), (16, 8, 2.0, 0.02, 3),
             (32, 16, 4.0, 0.05, 4), (24, 12, 3.0, 0.01, 6), (16, 8, 2.0, 0.02, 8)]
    for i, (n, nk, kr, dt, steps) in enumerate(specs):
        grid = inputs.cubic_grid(n, n * 0.5, nk, kr)
        jobs.append((grid, inputs.gaussian_field(grid, inputs.random_packets(3, 70 + i), dtype=torch.float32),
                     steps, dt))
    fs = [j[1].to(DEV) for j in jobs]
    advs = [chasm.Advect(f, j[0], 8, 6, j[3]) for f, j in zip(fs, jobs)]
    chasm.step_many(advs, [j[2] for j in jobs])
    torch.cuda.synchronize()
    for a in advs:
        a.close()
    for f, (grid, f0, steps, dt) in zip(fs, jobs):
        g = f0.to(DEV)
        with chasm.Advect(g, grid, 8, 6, dt) as a:
            a.step(steps)
        torch.cuda.synchronize()
        assert torch.equal(f, g)


def test_device_errors():
    w = inputs.workload("C1")
    cpu = torch.zeros(w.grid.shape(), dtype=torch.float32)
    d = chasm.make_desc(w.grid, w.patch, w.ghost, w.dt)
    with pytest.raises(chasm.ChasmError) as ei:
        chasm.chasm_advect_create(d, cpu.data_ptr(), 0)
    assert ei.value.status == chasm.CHASM_EINVAL
    buf = torch.zeros(w.grid.points + 4, dtype=torch.float32, device=DEV)
    with pytest.raises(chasm.ChasmError) as ei:
        chasm.chasm_advect_create(d, buf.data_ptr() + 4, 0)
    assert ei.value.status == chasm.CHASM_EINVAL
    f = torch.zeros(w.grid.shape(), dtype=torch.float32, device=DEV)
    with chasm.Advect(f, w.grid, w.patch, w.ghost, w.dt) as a:
        with pytest.raises(chasm.ChasmError) as ei:
            a.step(-1)
        assert ei.value.status == chasm.CHASM_EINVAL
        a.step(0)
        with pytest.raises(chasm.ChasmError):
            a.history()


# --------------------------------------------------------------------------- large grids
def _large_case(name, steps, nsample, seed, patch=None, ghost=None):
    import dataclasses
    w = inputs.workload(name)
    if patch is not None:
        w = dataclasses.replace(w, patch=(patch,) * 3, ghost=ghost)
    g = w.grid
    say(f"{name}: generating {g.points:.3e} points on the GPU")
    f = torch.empty(g.shape(), dtype=torch.float32, device=DEV)
    coef, gx, gk = inputs.packet_factors(g, w.packets)
    inputs.fill_separable(f, coef, gx, gk)
    kidx = inputs.k_sample(g, nsample / g.nkpts, seed)
    start = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    say(f"{name}: {steps} steps on the GPU")
    with chasm.Advect(f, g, w.patch, w.ghost, w.dt, graph=True) as a:
        sched = a.schedule
        a.step(steps)
    torch.cuda.synchronize()
    got = np.stack([f[i3, i2, i1].double().cpu().numpy() for i1, i2, i3 in kidx])
    say(f"{name}: oracle on {len(kidx)} sampled k-points")
    ref = oracle.advect6d(start, g.nx, g.hx, g.nk, g.k_lo, g.hk, w.patch, w.ghost, w.dt, steps, kidx=kidx)
    err = rel(got, ref)
    say(f"{name}: schedule={sched} sampled rel err {err:.3e}")
    assert err < 1e-4
    say(f"{name}: separable reference on every point")
    coef, U = oracle.separable_factors(g, w.packets, w.patch, w.ghost, w.dt, steps)
    ref_full = torch.empty(g.shape()[1:], dtype=torch.float32, device=DEV)
    worst, scale = 0.0, 0.0
    for i3 in range(g.nk[2]):
        # one k3 slab at a time keeps the reference small
        Us = [[U[p][0], U[p][1], U[p][2][i3:i3 + 1]] for p in range(len(coef))]
        sl = torch.empty((1,) + tuple(g.shape()[1:]), dtype=torch.float32, device=DEV)
        inputs.fill_separable(sl, coef, Us)
        worst = max(worst, float((f[i3] - sl[0]).abs().max()))
        scale = max(scale, float(sl.abs().max()))
    say(f"{name}: all points rel err {worst / scale:.3e}")
    assert worst / scale < 1e-4
    del f


def test_c3_slab_schedule_50_steps():
    """C3 over its 50 steps: 14 seeded k-points (1 per mille) against the oracle, every
    point against the separable reference."""
    _large_case("C3", 50, 14, 30)


@pytest.mark.parametrize("M", [8, 12])
@pytest.mark.parametrize("g", [4, 6, 8])
def test_c3_every_tuning_candidate(M, g):
    """The full 1.5e9-point C3 field under each (patch, ghost) the autotuner weighs
    (16/8 is the case above): all points against the separable reference."""
    _large_case("C3", 3, 2, 31, patch=M, ghost=g)


def test_c4_one_gpu_share_50_steps():
    """C4 over its 50 steps (graph-captured): a seeded 1 % sample of the k-points (328
    x-cubes of 64^3) against the FP64 oracle, every point against the separable
    reference."""
    _large_case("C4", 50, 328, 40)
