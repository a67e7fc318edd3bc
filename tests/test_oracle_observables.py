"""Pins of the observables oracle (Sec. 5's reduced Wigner functions and spatial
marginal): for one Gaussian packet pi^-3 exp(-|x-c|^2/s^2 - s^2 |k-k0|^2) inside the box
the integrals are closed forms,
  W_j(x, k) = pi^-1 exp(-(x-c_j)^2/s^2 - s^2 (k-k0_j)^2),
  P(x1, x2) = (pi s^2)^-1 exp(-((x1-c1)^2 + (x2-c2)^2)/s^2),
which the cell sums reproduce to rounding (trapezoid rule on a resolved Gaussian); each
observable integrates to the mass; an axis mix-up breaks the non-cubic-grid case."""
import math

import numpy as np

from oracle import observables
from paper_2205_02380_amd import inputs


def test_gaussian_packet_closed_forms():
    grid = inputs.Grid((24, 20, 16), (-7.0, -6.0, -5.0), (7.0, 6.0, 5.0), (12, 14, 16),
                       (-4.8, -5.0, -5.6), (4.8, 5.0, 5.6))
    c, k0, s = (0.4, -0.3, 0.2), (0.3, -0.2, 0.5), 1.1
    pk = inputs.Packets(w=np.array([1.0]), c=np.array([c]), k0=np.array([k0]), s=np.array([s]))
    f = inputs.gaussian_field(grid, pk).numpy()
    w1, w2, w3, p = observables.marginals(f, grid.hx, grid.hk)
    # 1-D cell sums of the packet's factors: the discrete integrals factorise exactly
    sx = [np.sum(np.exp(-(grid.x_axis(d) - c[d]) ** 2 / s ** 2)) * grid.hx[d] for d in range(3)]
    sk = [np.sum(np.exp(-s ** 2 * (grid.k_axis(d) - k0[d]) ** 2)) * grid.hk[d] for d in range(3)]
    for d, w in enumerate((w1, w2, w3)):
        x, k = grid.x_axis(d), grid.k_axis(d)
        g = np.exp(-(x[None, :] - c[d]) ** 2 / s ** 2 - s ** 2 * (k[:, None] - k0[d]) ** 2)
        o = [e for e in range(3) if e != d]
        exact_sum = g * math.pi ** -3 * sx[o[0]] * sx[o[1]] * sk[o[0]] * sk[o[1]]
        assert w.shape == g.shape
        assert np.max(np.abs(w - exact_sum)) < 1e-12 * np.max(exact_sum), d
        # and the integral's closed form, to the trapezoid/truncation error of this grid
        assert np.max(np.abs(w - g / math.pi)) < 1e-5 * np.max(g / math.pi), d
    x1, x2 = grid.x_axis(0), grid.x_axis(1)
    g = np.exp(-((x1[None, :] - c[0]) ** 2 + (x2[:, None] - c[1]) ** 2) / s ** 2)
    exact_sum = g * math.pi ** -3 * sx[2] * sk[0] * sk[1] * sk[2]
    assert np.max(np.abs(p - exact_sum)) < 1e-12 * np.max(exact_sum)
    assert np.max(np.abs(p - g / (math.pi * s * s))) < 1e-5 * np.max(g) / (math.pi * s * s)


def test_observables_integrate_to_the_mass_with_batch():
    grid = inputs.Grid((8, 6, 10), (-3.0,) * 3, (3.0,) * 3, (4, 5, 3), (-2.0,) * 3, (2.0,) * 3)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((2,) + grid.shape())
    mass = f.reshape(2, -1).sum(axis=1) * np.prod(grid.hx) * np.prod(grid.hk)
    w1, w2, w3, p = observables.marginals(f, grid.hx, grid.hk)
    for d, w in enumerate((w1, w2, w3)):
        assert w.shape == (2, grid.nk[d], grid.nx[d])
        assert np.allclose(w.sum(axis=(1, 2)) * grid.hx[d] * grid.hk[d], mass, rtol=1e-12)
    assert p.shape == (2, grid.nx[1], grid.nx[0])
    assert np.allclose(p.sum(axis=(1, 2)) * grid.hx[0] * grid.hx[1], mass, rtol=1e-12)
