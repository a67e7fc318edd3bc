"""Out-of-place sweeps (a library-owned stage field): the arithmetic is the same as in
place, so every result must equal the in-place run bitwise, for every schedule, step
count parity (CUBE runs pairs of steps through the stage field), graph replay, the
per-step diagnostics history and batched stepping of mixed handles."""
import numpy as np
import pytest
import torch

import oracle
from paper_2205_02380_amd import chasm, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _field(grid, seed, dtype=torch.float32):
    return inputs.gaussian_field(grid, inputs.random_packets(3, seed), dtype=dtype)


def _run(f0, grid, M, g, dt, steps, **kw):
    f = f0.to(DEV)
    with chasm.Advect(f, grid, M, g, dt, **kw) as a:
        a.step(steps)
        hist = a.history() if kw.get("reduce_each_step") else None
    torch.cuda.synchronize()
    return f, hist


CASES = [  # (N, M, g, nk, schedules)
    (32, 16, 4, 6, ("cube", "slab", "plain")),
    (48, 12, 6, 4, ("slab", "plain")),
]


@pytest.mark.parametrize("N,M,g,nk,scheds", CASES)
@pytest.mark.parametrize("steps", [1, 2, 3, 5, 19])
def test_out_of_place_equals_in_place(N, M, g, nk, scheds, steps):
    grid = inputs.cubic_grid(N, N * 0.4, nk, 3.0)
    dt = 0.45
    f0 = _field(grid, 900 + N + steps)
    for sched in scheds:
        for graph in (False, True):
            print(f"N={N} M={M} g={g} {sched} steps={steps} graph={graph}", flush=True)
            ref, href = _run(f0, grid, M, g, dt, steps, schedule=sched, graph=graph, reduce_each_step=True)
            out, hout = _run(f0, grid, M, g, dt, steps, schedule=sched, graph=graph, reduce_each_step=True,
                             out_of_place=True)
            assert torch.equal(ref, out), (sched, graph)
            assert np.array_equal(href, hout), (sched, graph)


def test_out_of_place_matches_oracle_fp64():
    """Ties the stage path to the oracle directly: FP64, CUBE pairs and an odd tail."""
    grid = inputs.cubic_grid(16, 6.4, 4, 2.0)
    f0 = _field(grid, 77, torch.float64)
    ref = oracle.advect6d(f0.numpy(), grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, (8,) * 3, 4, 0.3, 3)
    for sched in ("cube", "slab", "plain"):
        if not chasm.supported(grid, 8, 4, 0.3, "f64", "pmbc", sched):
            continue
        out, _ = _run(f0, grid, 8, 4, 0.3, 3, schedule=sched, out_of_place=True)
        err = float(np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref)))
        assert err < 1e-12, (sched, err)


def test_step_many_mixes_in_place_and_out_of_place_handles():
    """Handles of one shape share launches whatever their placement; each equals its
    solo in-place run."""
    specs = [(32, 0.02, 5, False), (32, 0.05, 4, True), (32, 0.03, 3, True), (48, 0.02, 2, True),
             (48, 0.04, 3, False)]
    fs, advs, solo = [], [], []
    for i, (n, dt, steps, oop) in enumerate(specs):
        grid = inputs.cubic_grid(n, n * 0.5, 4, 2.0)
        f0 = _field(grid, 300 + i)
        M, g = (16, 4) if n == 32 else (12, 6)
        sched = "slab"
        f = f0.to(DEV)
        fs.append(f)
        advs.append(chasm.Advect(f, grid, M, g, dt, schedule=sched, out_of_place=oop))
        solo.append(_run(f0, grid, M, g, dt, steps, schedule=sched)[0])
    chasm.step_many(advs, [s[2] for s in specs])
    torch.cuda.synchronize()
    for a in advs:
        a.close()
    for f, r in zip(fs, solo):
        assert torch.equal(f, r)


def test_reversed_visiting_order_is_bitwise_neutral():
    """chasm_advect_step alternates the CUBE item order between steps; chasm_advect_step_many
    always visits forward.  Fields and per-step diagnostics agree bitwise."""
    grid = inputs.cubic_grid(32, 12.8, 6, 3.0)
    f0 = _field(grid, 4242)
    fa, fb = f0.to(DEV), f0.to(DEV)
    with chasm.Advect(fa, grid, 16, 4, 0.45, schedule="cube", reduce_each_step=True) as a, \
            chasm.Advect(fb, grid, 16, 4, 0.45, schedule="cube", reduce_each_step=True, graph=True) as b:
        for _ in range(5):
            chasm.step_many([a], [1])          # forward order every step
        b.step(5)                               # forward, reverse, forward, ...
        torch.cuda.synchronize()
        ha, hb = a.history(), b.history()
    assert torch.equal(fa, fb)
    assert np.array_equal(ha, hb)
