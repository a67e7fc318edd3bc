"""Every compiled kernel shape (dtype, N, M, ghost, closure: the paper's PMBC, its
Neumann-condition variant and the cubic-exact variant) against the FP64 oracle,
under every schedule the shape supports, on a small ragged k grid whose shifts take
both signs, zero and |alpha| > 1.  This covers each candidate the autotuner may pick
(C3: N = 48, M in {8, 12, 16}, g in {4, 6, 8}; C4: N = 64, M in {8, 16}, g in {4, 6, 8})."""
import numpy as np
import pytest
import torch

import oracle
from paper_2205_02380_amd import chasm, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

try:
    SHAPES = chasm.compiled_shapes()
except RuntimeError:          # library not built: nothing to collect
    SHAPES = []


def small_grid(n):
    h, hk = 0.5, 0.5
    nk = (4, 3, 2)
    return inputs.Grid((n, n, n), (-n * h / 2,) * 3, (n * h / 2,) * 3, nk,
                       tuple(-hk * (m // 2) for m in nk), tuple(hk * (m - m // 2) for m in nk))


@pytest.mark.parametrize("dtype,N,M,g,closure", SHAPES)
def test_compiled_shape_matches_oracle(dtype, N, M, g, closure):
    grid = small_grid(N)
    dt = 1.15                       # alpha = k dt / h: k1 = -2 hk gives alpha = -2.3
    pk = inputs.random_packets(2, 100 * N + 10 * M + g, c_range=(-1.0, 1.0), s_range=(0.6, 1.0))
    f0 = inputs.gaussian_field(grid, pk).numpy()
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    steps = 2
    cl = {"pmbc": oracle.PMBC, "poly3": oracle.POLY3, "neumann": oracle.NEUMANN}[closure]
    ref = oracle.advect6d(f0, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, (M,) * 3, g, dt, steps, closure=cl)
    tol = 1e-5 if dtype == "f32" else (1e-10 if closure == "poly3" else 1e-12)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    scale = np.max(np.abs(ref))
    ran = []
    for sched in ("cube", "slab", "plain"):
        if not chasm.supported(grid, M, g, dt, dtype, closure, sched):
            continue
        print(f"shape {dtype} N={N} M={M} g={g} {closure} {sched}", flush=True)
        f = torch.tensor(f0, dtype=tdt, device=DEV)
        with chasm.Advect(f, grid, M, g, dt, closure=closure, schedule=sched) as a:
            a.step(steps)
        torch.cuda.synchronize()
        err = float(np.max(np.abs(f.double().cpu().numpy() - ref))) / scale
        assert err < tol, (sched, err)
        ran.append(sched)
    assert "slab" in ran and "plain" in ran
