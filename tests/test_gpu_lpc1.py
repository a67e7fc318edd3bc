"""GPU parity of the LPC1 step (Sec. 2.2: characteristic step + truncated-kernel
Theta_V, predictor and corrector in the library's kernels) against the FP64 oracle
composition.  FP64 fields: <= 1e-11 of max|f| after 3 steps; FP32: <= 1e-5."""
import numpy as np
import pytest
import torch

from oracle import lpc1 as olpc1
from paper_2205_02380_amd import chasm, inputs, lpc1

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
H2 = [(-0.614161, 0.0, 0.0), (0.614161, 0.0, 0.0)]


def field(grid, seed):
    pk = inputs.random_packets(2, seed, c_range=(-1.0, 1.0), k0_range=(-0.5, 0.5), s_range=(0.8, 1.1))
    return inputs.gaussian_field(grid, pk).numpy()


@pytest.mark.parametrize("dtype,steps,tol", [("f64", 3, 1e-11), ("f32", 3, 1e-5)])
def test_lpc1_matches_oracle_nk8(dtype, steps, tol):
    grid = inputs.Grid((8, 8, 8), (-3.0,) * 3, (3.0,) * 3, (8, 8, 8), (-2.4,) * 3, (2.4,) * 3)
    f0 = field(grid, 5)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    f = torch.tensor(f0, dtype=tdt, device=DEV)
    start = f.double().cpu().numpy()
    print(f"lpc1 nk=8 {dtype} {steps} steps", flush=True)
    with lpc1.LPC1(f, grid, 4, 3, 0.05, [(0.2, -0.1, 0.3)], [1.0]) as s:
        s.step(steps)
    torch.cuda.synchronize()
    ref = olpc1.lpc1(start, grid, 4, 3, 0.05, steps, [(0.2, -0.1, 0.3)], [1.0])
    got = f.double().cpu().numpy()
    assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref))
    assert np.max(np.abs(got - start)) > 1e-3 * np.max(np.abs(start))    # it moved


def test_lpc1_two_protons_nk16_one_step():
    grid = inputs.Grid((8, 8, 8), (-3.0,) * 3, (3.0,) * 3, (16, 16, 16), (-4.0,) * 3, (4.0,) * 3)
    f0 = field(grid, 6)
    f = torch.tensor(f0, dtype=torch.float64, device=DEV)
    print("lpc1 nk=16 H2 one step", flush=True)
    with lpc1.LPC1(f, grid, 4, 3, 0.025, H2) as s:
        s.step(1)
    torch.cuda.synchronize()
    ref = olpc1.lpc1(f0, grid, 4, 3, 0.025, 1, H2, [1.0, 1.0], direct=False)
    assert np.max(np.abs(f.cpu().numpy() - ref)) < 1e-11 * np.max(np.abs(ref))


def test_lpc1_without_potential_is_the_advection_bitwise():
    grid = inputs.Grid((16, 16, 16), (-6.0,) * 3, (6.0,) * 3, (8, 8, 8), (-2.4,) * 3, (2.4,) * 3)
    f0 = field(grid, 7)
    f = torch.tensor(f0, dtype=torch.float32, device=DEV)
    g = f.clone()
    with lpc1.LPC1(f, grid, 8, 4, 0.05, [(0.0, 0.0, 0.0)], [0.0]) as s:
        s.step(4)
    with chasm.Advect(g, grid, 8, 4, 0.05) as a:             # the step advects the caller's field in place
        a.step(4)
    torch.cuda.synchronize()
    assert torch.equal(f, g)


def test_lpc1_rejects_mismatched_descriptors():
    grid = inputs.Grid((8, 8, 8), (-3.0,) * 3, (3.0,) * 3, (8, 8, 8), (-2.4,) * 3, (2.4,) * 3)
    f = torch.zeros(grid.shape(), dtype=torch.float32, device=DEV)
    from paper_2205_02380_amd import theta
    adv = chasm.make_desc(grid, 4, 3, 0.05)
    other = inputs.Grid((8, 8, 8), (-3.0,) * 3, (3.0,) * 3, (8, 8, 8), (-2.0,) * 3, (2.4,) * 3)
    th = theta.make_desc(other, [(0.0, 0.0, 0.0)])
    with pytest.raises(chasm.ChasmError) as ei:
        lpc1.chasm_lpc1_create(adv, th, f.data_ptr(), 0)
    assert ei.value.status == chasm.CHASM_EINVAL
    s = lpc1.LPC1(f, grid, 4, 3, 0.05, [(0.0, 0.0, 0.0)])
    with pytest.raises(chasm.ChasmError):
        s.step(-1)
    s.close()


def test_lpc1_on_a_runtime_shape_grid():
    """An anisotropic x-grid without compiled advection kernels: the LPC1 step's
    characteristic step runs on the runtime-shape kernels."""
    grid = inputs.Grid((9, 7, 6), (-3.0, -2.5, -2.0), (3.0, 2.5, 2.0), (8, 8, 8), (-2.4,) * 3, (2.4,) * 3)
    f0 = field(grid, 8)
    f = torch.tensor(f0, dtype=torch.float64, device=DEV)
    print("lpc1 runtime-shape grid 9x7x6, nk=8, 2 steps", flush=True)
    with lpc1.LPC1(f, grid, (4, 3, 5), 3, 0.05, [(0.2, -0.1, 0.3)], [1.0]) as s:
        s.step(2)
    torch.cuda.synchronize()
    ref = olpc1.lpc1(f0, grid, (4, 3, 5), 3, 0.05, 2, [(0.2, -0.1, 0.3)], [1.0])
    assert np.max(np.abs(f.cpu().numpy() - ref)) < 1e-11 * np.max(np.abs(ref))


def test_lpc1_nk32_staged_theta_on_the_paper_patch_line():
    """N_k = 32 (the staged Theta_V) on an x-grid of 16 x 2 x 2 nodes whose first axis
    has the paper's patch and ghost width (one patch of 15 cells, n_nb = 15: the unrolled
    runtime-shape form), one step, FP64, against the oracle (threefold transforms)."""
    grid = inputs.Grid((16, 2, 2), (-2.4, -0.3, -0.3), (2.4, 0.3, 0.3), (32, 32, 32), (-6.4,) * 3, (6.4,) * 3)
    f0 = field(grid, 9)
    f = torch.tensor(f0, dtype=torch.float64, device=DEV)
    nuclei = [(0.35, 0.05, -0.1)]
    print("lpc1 16x2x2 x 32^3, one step", flush=True)
    with lpc1.LPC1(f, grid, (15, 1, 1), 15, 0.025, nuclei, [1.0]) as s:
        s.step(1)
    torch.cuda.synchronize()
    print("  oracle", flush=True)
    ref = olpc1.lpc1(f0, grid, (15, 1, 1), 15, 0.025, 1, nuclei, [1.0], direct=False)
    err = float(np.max(np.abs(f.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    print(f"  rel err {err:.2e}", flush=True)
    assert err < 1e-11
