"""GPU parity of the 2-D harmonic-oscillator workload (Sec. 5.1: LPC1 with the
patched-spline x-advection and the spectral k-derivative) against the FP64 oracle, and
its accuracy against the exact phase-space rotation over one full period."""
import math

import numpy as np
import pytest
import torch

from oracle import ho2d as oho
from paper_2205_02380_amd import ho2d

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
W = (math.pi / 5.0) ** 2


def run(nx, hx, nk, hk, M, g, tau, steps, inflow="zero"):
    x, k = oho.axes(nx, -12.0, hx, nk, -nk * hk / 2, hk)
    f0 = oho.f0(x[None, :], k[:, None])
    f = torch.tensor(f0, dtype=torch.float64, device=DEV)
    with ho2d.HO2D(f, nx, -12.0, hx, nk, -nk * hk / 2, hk, M, g, W, tau, inflow=inflow) as s:
        s.step(steps)
    torch.cuda.synchronize()
    return x, k, f0, f.cpu().numpy()


@pytest.mark.parametrize("inflow", ["zero", "extrapolate"])
@pytest.mark.parametrize("nx,hx,nk,hk,M,g,tau,steps", [
    (121, 0.2, 128, 0.1, 30, 20, 0.005, 10),
    (241, 0.1, 512, 0.025, 60, 20, 0.00002, 5),         # the paper's grid and time step
    (61, 0.4, 64, 0.2, 16, 6, 0.01, 8),                   # ragged last patch (60 = 3 x 16 + 12)
    (121, 0.2, 256, 0.05, 30, 20, 0.004, 6),              # transform path 16 x 16
    (121, 0.2, 1024, 0.0125, 30, 20, 0.002, 4),           # transform path 32 x 32
    (81, 0.3, 96, 0.1, 20, 10, 0.005, 6),                 # nk not a power of two: dense path
    (41, 0.6, 2048, 0.00625, 10, 6, 0.001, 3),            # nk above the transform sizes: dense path
])
def test_ho2d_matches_oracle(nx, hx, nk, hk, M, g, tau, steps, inflow):
    print(f"ho2d nx={nx} nk={nk} steps={steps} inflow={inflow}", flush=True)
    x, k, f0, got = run(nx, hx, nk, hk, M, g, tau, steps, inflow)
    ref = oho.lpc1(f0, x, k, hx, hk, M, g, W, tau, steps, inflow)
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


def test_ho2d_full_period_returns_to_the_start():
    """T = 10 is one period for omega = (pi/5)^2: 10000 LPC1 steps of tau = 1e-3 on
    dx = 0.2 (121 nodes, 4 patches, n_nb = 20), dk = 0.1; the packet returns to its start
    (measured eps_inf(10) = 1.65e-4) and the mass is kept to rounding."""
    print("ho2d full period", flush=True)
    x, k, f0, got = run(121, 0.2, 128, 0.1, 30, 20, 0.001, 10000)
    ex = oho.exact(x, k, 10.0, W)
    err = np.max(np.abs(got - ex))
    mass0, mass = f0.sum() * 0.2 * 0.1, got.sum() * 0.2 * 0.1
    print(f"eps_inf(10) = {err:.3e}, mass deviation {abs(mass - mass0):.3e}", flush=True)
    assert err < 3e-4
    assert abs(mass - mass0) < 1e-10


def test_ho2d_paper_grid_to_t6_extrapolated_inflow():
    """The paper's grid and step (dx = 0.1, dk = 0.025, tau = 2e-5) up to t = 6 (300000
    steps) with ghost-extrapolated inflow: eps_inf stays at the 5e-6 level.  (Beyond
    t ~ 6.4 a mode at the x = 12 boundary column, grown from rounding at ~e^4.1 per unit
    time, takes over in this mode; zero inflow, the default, stays stable to T = 10 --
    measured by the benchmark.)"""
    print("ho2d paper grid to t = 6", flush=True)
    x, k, f0, got = run(241, 0.1, 512, 0.025, 60, 20, 0.00002, 300000, "extrapolate")
    err = np.max(np.abs(got - oho.exact(x, k, 6.0, W)))
    print(f"eps_inf(6) = {err:.3e}", flush=True)
    assert err < 1e-5
