"""GPU: the autotuner's tile-shape axis.

* The launch-shape variants of the SLAB and PLAIN passes (x3-slabs per slab block,
  lines per pencil block) leave each line's arithmetic unchanged: the fields are
  bitwise equal to the default shape's, and the fused FP64 reductions (eq. 2.5
  diagnostics of Sec. 5, one history row per step) equal the oracle's sums of the
  stored field to 1e-12; sampled k-points match the FP64 oracle to 1e-5.
* ``autotune.tune()`` over patch x ghost x schedule x tile x placement on a small
  48^3 grid: the winner's field matches the oracle at its own (patch, ghost) to 1e-5
  and the oracle at the most accurate candidate (patch 16, ghost 8) within the tuner's
  tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2205_02380_amd import autotune, chasm, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def grid_of(N, nk):
    return inputs.Grid((N,) * 3, (-N / 4.0,) * 3, (N / 4.0,) * 3, nk, (-2.0,) * 3, (1.8,) * 3)


@pytest.mark.parametrize("N,M,g,nk", [(48, 12, 6, (2, 2, 1)), (48, 16, 8, (2, 1, 2)), (64, 16, 8, (2, 1, 1))])
@pytest.mark.parametrize("schedule", ["slab", "plain"])
def test_tile_variants_bitwise_equal_and_reductions_match_oracle(N, M, g, nk, schedule):
    grid = grid_of(N, nk)
    pk = inputs.random_packets(3, 800 + N + M, c_range=(-N / 8.0, N / 8.0), k0_range=(-0.5, 0.5), s_range=(0.8, 1.4))
    f0 = inputs.gaussian_field(grid, pk, dtype=torch.float32)
    dt = 0.05
    outs = []
    for tile in (0, 1, 2):
        say(f"N={N} M={M} g={g} {schedule} tile {tile}")
        f = f0.to(DEV)
        with chasm.Advect(f, grid, M, g, dt, schedule=schedule, reduce_each_step=True, tile=tile) as a:
            assert a.schedule == schedule
            expect = []
            for _ in range(3):          # one step per call: every history row is a stored field
                a.step(1)
                torch.cuda.synchronize()
                expect.append(oracle.reduce(f.double().cpu().numpy(), grid.nx, grid.x_lo, grid.hx, grid.nk,
                                            grid.k_lo, grid.hk))
            hist = a.history()
        for s in range(3):
            for i in range(8):
                assert hist[s, 0, i] == pytest.approx(expect[s][i], rel=1e-12, abs=1e-14 * abs(expect[s][0]) * 16)
        outs.append(f.cpu())
    assert torch.equal(outs[1], outs[0]) and torch.equal(outs[2], outs[0])
    kidx = inputs.k_sample(grid, 2 / grid.nkpts, 7)
    start = np.stack([f0[i3, i2, i1].double().numpy() for i1, i2, i3 in kidx])
    ref = oracle.advect6d(start, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, (M,) * 3, g, dt, 3, kidx=kidx)
    got = np.stack([outs[0][i3, i2, i1].double().numpy() for i1, i2, i3 in kidx])
    assert np.max(np.abs(got - ref)) < 1e-5 * np.max(np.abs(ref))


def test_tune_on_a_small_48_grid():
    grid = inputs.Grid((48,) * 3, (-16.0,) * 3, (16.0,) * 3, (2, 2, 2), (-4.0,) * 3, (4.0,) * 3)
    pk = inputs.random_packets(4, 77)
    dt, tol = 0.02, 1e-5
    res = autotune.tune(grid, dt, pk, schedules=("slab", "plain"), steps=3, warmup=1, tol=tol, log=say,
                        reduce_each_step=True)             # timed as the benchmark runs them
    cands, best = res["candidates"], res["best"]
    assert res["reduce_each_step"]
    assert len(cands) == 9 * 2 * 3 * 2 and {c["tile"] for c in cands} == {0, 1, 2}
    assert best["ok"] and best["deviation"] <= tol
    say(f"winner: {best}")
    f = inputs.gaussian_field(grid, pk, dtype=torch.float32).to(DEV)
    start = f.double().cpu().numpy()
    with chasm.Advect(f, grid, best["patch"], best["ghost"], dt, schedule=best["schedule"], tile=best["tile"],
                      out_of_place=best["out_of_place"]) as a:
        a.step(3)
    torch.cuda.synchronize()
    got = f.double().cpu().numpy()
    own = oracle.advect6d(start, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, (best["patch"],) * 3, best["ghost"],
                          dt, 3)
    ref = oracle.advect6d(start, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, (16,) * 3, 8, dt, 3)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - own)) <= 1e-5 * scale
    assert np.max(np.abs(got - ref)) <= (tol + 1e-5) * scale
