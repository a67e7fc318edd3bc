"""Pins of the LPC1 oracle (Sec. 2.2) beyond its component operators' own pins:
* Theta = 0 (no nuclei, or zero charge): a step is exactly the characteristic step;
* tau -> 0: (step - characteristic step) / tau -> Theta[f], with an error that halves
  with tau (first order), which fixes the tau and tau/2 coefficients of the predictor and
  corrector (a wrong coefficient leaves an O(1) gap);
* linearity in f.
"""
import numpy as np

from oracle import lpc1
from paper_2205_02380_amd import inputs

GRID = inputs.Grid((6, 5, 4), (-3.0, -2.5, -2.0), (3.0, 2.5, 2.0), (6, 6, 6), (-2.4,) * 3, (2.4,) * 3)
M, G = 3, 2
NUC = [(0.2, -0.1, 0.3)]


def field(seed):
    pk = inputs.random_packets(2, seed, c_range=(-1.0, 1.0), k0_range=(-0.5, 0.5), s_range=(0.8, 1.1))
    return inputs.gaussian_field(GRID, pk).numpy()


def test_no_potential_is_the_characteristic_step():
    f = field(1)
    a = lpc1.lpc1(f, GRID, M, G, 0.1, 2, NUC, [0.0])
    b = lpc1.advect(lpc1.advect(f, GRID, M, G, 0.1), GRID, M, G, 0.1)
    assert np.max(np.abs(a - b)) == 0.0


def test_small_tau_limit_is_theta():
    f = field(2)
    th = lpc1.theta_field(f, GRID, NUC, [1.0])
    gaps = []
    for tau in (4e-3, 2e-3, 1e-3):
        d = (lpc1.lpc1(f, GRID, M, G, tau, 1, NUC, [1.0]) - lpc1.advect(f, GRID, M, G, tau)) / tau
        gaps.append(np.max(np.abs(d - th)) / np.max(np.abs(th)))
    assert gaps[-1] < 0.02
    assert 1.7 < gaps[0] / gaps[1] < 2.3 and 1.7 < gaps[1] / gaps[2] < 2.3


def test_linear_in_f():
    f, g = field(3), field(4)
    a = lpc1.lpc1(2.0 * f - 0.5 * g, GRID, M, G, 0.05, 1, NUC, [1.0])
    b = 2.0 * lpc1.lpc1(f, GRID, M, G, 0.05, 1, NUC, [1.0]) - 0.5 * lpc1.lpc1(g, GRID, M, G, 0.05, 1, NUC, [1.0])
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))
