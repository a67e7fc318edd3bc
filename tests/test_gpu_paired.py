"""The SLAB schedule's alternating sweep order (x1 x2 x3, then x3 x2 x1, ...; K steps
in K + 1 passes) against the FP64 oracle, which always sweeps x1, x2, x3.  The axis
operators of the tensor-product spline (eqs. 3.11-3.12) commute, so the two orders
agree up to rounding.  Also: graph replay equals eager issue bitwise for the same
step counts, and step_many with SLAB handles of different step counts equals each
handle run alone, bitwise (the pass sequence of a handle depends only on its K)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2205_02380_amd import chasm, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def _grid(N, nk, kr):
    return inputs.Grid((N,) * 3, (-N / 4.0,) * 3, (N / 4.0,) * 3, nk, (-kr,) * 3, (kr * 0.9,) * 3)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 8, 9, 10, 13])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_slab_any_step_count_matches_oracle(K, dtype):
    grid = _grid(16, (4, 3, 2), 2.0)
    dt = 0.35                                  # |alpha| up to 1.4: shift classes 0, -1 and others
    f0 = inputs.gaussian_field(grid, inputs.random_packets(3, 500 + K, c_range=(-1.5, 1.5))).numpy()
    start = f0.astype(np.float32).astype(np.float64) if dtype == torch.float32 else f0
    say(f"slab K={K} {dtype}")
    f = torch.tensor(start, dtype=dtype, device=DEV)
    with chasm.Advect(f, grid, 8, 4, dt, schedule="slab") as a:
        a.step(K)
    torch.cuda.synchronize()
    ref = oracle.advect6d(start, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, (8, 8, 8), 4, dt, K)
    err = float(np.max(np.abs(f.double().cpu().numpy() - ref)) / np.max(np.abs(ref)))
    say(f"  rel err {err:.2e}")
    assert err < (1e-12 * max(K, 1) if dtype == torch.float64 else 1e-5 * max(1, K / 10))


@pytest.mark.parametrize("N,M,g", [(48, 16, 8), (64, 16, 8), (48, 8, 4)])
def test_slab_large_lines_match_oracle(N, M, g):
    grid = _grid(N, (2, 2, 2), 3.0)
    dt = 0.2
    f0 = inputs.gaussian_field(grid, inputs.random_packets(3, 520 + N, c_range=(-N / 8, N / 8))).numpy()
    start = f0.astype(np.float32).astype(np.float64)
    for K in (1, 2, 3, 6):
        say(f"slab N={N} M={M} g={g} K={K}")
        f = torch.tensor(start, dtype=torch.float32, device=DEV)
        with chasm.Advect(f, grid, M, g, dt, schedule="slab", graph=True) as a:
            a.step(K)
        torch.cuda.synchronize()
        ref = oracle.advect6d(start, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, (M,) * 3, g, dt, K)
        err = float(np.max(np.abs(f.double().cpu().numpy() - ref)) / np.max(np.abs(ref)))
        say(f"  rel err {err:.2e}")
        assert err < 1e-5


def test_slab_graph_equals_eager_bitwise():
    grid = _grid(32, (4, 4, 2), 2.0)
    f0 = inputs.gaussian_field(grid, inputs.random_packets(3, 540), dtype=torch.float32)
    a_out, b_out = f0.to(DEV), f0.to(DEV)
    calls = [1, 2, 3, 11, 20, 4]               # every graph of the pass sequences is used
    with chasm.Advect(a_out, grid, 8, 6, 0.05, schedule="slab") as a, \
            chasm.Advect(b_out, grid, 8, 6, 0.05, schedule="slab", graph=True) as b:
        for k in calls:
            a.step(k)
            b.step(k)
    torch.cuda.synchronize()
    assert torch.equal(a_out, b_out)


def test_slab_out_of_place_equals_in_place_bitwise():
    grid = _grid(32, (3, 2, 2), 2.0)
    f0 = inputs.gaussian_field(grid, inputs.random_packets(2, 545), dtype=torch.float32)
    for graph in (False, True):
        a_out, b_out = f0.to(DEV), f0.to(DEV)
        with chasm.Advect(a_out, grid, 8, 6, 0.1, schedule="slab", graph=graph, reduce_each_step=True) as a, \
                chasm.Advect(b_out, grid, 8, 6, 0.1, schedule="slab", graph=graph, reduce_each_step=True,
                             out_of_place=True) as b:
            for k in (1, 2, 5, 12):
                a.step(k)
                b.step(k)
            ha, hb = a.history(), b.history()
        torch.cuda.synchronize()
        assert torch.equal(a_out, b_out), graph
        assert np.array_equal(ha, hb), graph


def test_step_many_slab_handles_equal_solo_runs():
    specs = [(32, 4, 0.02, 5), (32, 4, 0.05, 2), (48, 2, 0.02, 7), (32, 4, 0.03, 1), (48, 2, 0.04, 4),
             (32, 4, 0.02, 0), (32, 4, 0.01, 6)]
    jobs = []
    for i, (n, nk, dt, steps) in enumerate(specs):
        grid = inputs.cubic_grid(n, n * 0.5, nk, 2.0)
        jobs.append((grid, inputs.gaussian_field(grid, inputs.random_packets(2, 560 + i), dtype=torch.float32),
                     steps, dt))
    fs = [j[1].to(DEV) for j in jobs]
    advs = [chasm.Advect(f, j[0], 8, 6, j[3], schedule="slab") for f, j in zip(fs, jobs)]
    chasm.step_many(advs, [j[2] for j in jobs])
    torch.cuda.synchronize()
    for a in advs:
        a.close()
    for f, (grid, f0, steps, dt) in zip(fs, jobs):
        g = f0.to(DEV)
        with chasm.Advect(g, grid, 8, 6, dt, schedule="slab") as a:
            a.step(steps)
        torch.cuda.synchronize()
        assert torch.equal(f, g)
