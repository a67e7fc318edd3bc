"""Pins of the 2-D harmonic-oscillator oracle (Sec. 5.1), against what mathematics fixes:
the spectral k-derivative of band-limited periodic data is exact; with omega = 0 the
scheme is the characteristic step (free streaming); the LPC1 solution follows the exact
phase-space rotation of eq. 5.2 with an error that falls when dx and tau are refined;
the total mass is conserved to the PMBC truncation level."""
import math

import numpy as np

from oracle import ho2d

W = (math.pi / 5.0) ** 2           # the example's omega: period T = 10


def test_spectral_derivative_exact_on_band_limited_data():
    n, hk = 64, 0.2
    L = n * hk
    k = -L / 2 + hk * np.arange(n)
    f = np.sin(2 * math.pi * 3 * k / L)[:, None] * np.array([1.0, -2.0])[None, :]
    d = ho2d.dk_spectral(f, hk)
    ex = (2 * math.pi * 3 / L) * np.cos(2 * math.pi * 3 * k / L)[:, None] * np.array([1.0, -2.0])[None, :]
    assert np.max(np.abs(d - ex)) < 1e-12


def test_zero_frequency_is_the_characteristic_step():
    x, k = ho2d.axes(41, -6.0, 0.3, 32, -3.2, 0.2)
    f = ho2d.f0(x[None, :], k[:, None])
    a = ho2d.lpc1(f, x, k, 0.3, 0.2, 10, 8, 0.0, 0.05, 2)
    b = ho2d.advect(ho2d.advect(f, x, k, 0.3, 10, 8, 0.05), x, k, 0.3, 10, 8, 0.05)
    assert np.max(np.abs(a - b)) == 0.0


def _err(nx, hx, tau, t_end):
    x, k = ho2d.axes(nx, -12.0, hx, 128, -6.4, 0.1)
    f = ho2d.f0(x[None, :], k[:, None])
    M = (nx - 1) // 4
    n = int(round(t_end / tau))
    got = ho2d.lpc1(f, x, k, hx, 0.1, M, 20, W, tau, n)
    ex = ho2d.exact(x, k, n * tau, W)
    mass0, mass = f.sum() * hx * 0.1, got.sum() * hx * 0.1
    return np.max(np.abs(got - ex)), abs(mass - mass0)


def test_follows_the_exact_rotation_and_conserves_mass():
    e1, m1 = _err(61, 0.4, 0.01, 0.5)
    e2, m2 = _err(121, 0.2, 0.005, 0.5)
    # halving dx and tau together: 13x smaller here (4th order in dx, 2nd in tau, Sec. 5.1)
    assert e2 < 1e-5 and e2 < e1 / 8
    # the paper reports a mass loss of about 1e-13 with the natural condition and n_nb >= 20
    assert m1 < 1e-12 and m2 < 1e-12


def test_inflow_modes_differ_only_at_inflow_nodes():
    """Zero inflow sets exactly the nodes whose departure point leaves [x_0, x_{N-1}] to 0
    (the right end for k < 0, the left end for k > 0); elsewhere it equals the
    ghost-extrapolating step bitwise."""
    x, k = ho2d.axes(41, -6.0, 0.3, 16, -3.2, 0.4)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((16, 41))
    tau = 0.05
    z = ho2d.advect(f, x, k, 0.3, 10, 8, tau, inflow="zero")
    e = ho2d.advect(f, x, k, 0.3, 10, 8, tau, inflow="extrapolate")
    for i, kv in enumerate(k):
        if kv < 0:
            assert z[i, -1] == 0.0 and e[i, -1] != 0.0
            assert np.array_equal(z[i, :-1], e[i, :-1])
        elif kv > 0:
            assert z[i, 0] == 0.0 and e[i, 0] != 0.0
            assert np.array_equal(z[i, 1:], e[i, 1:])
        else:
            assert np.array_equal(z[i], e[i]) and np.allclose(z[i], f[i], rtol=0, atol=1e-13)


def _one_step_matrix(nx, x_lo, hx, nk, k_lo, hk, M, g, omega, tau, inflow):
    """The LPC1 step of the oracle as a matrix on the state f[k][x] (row-major): with
    A the characteristic step (block-diagonal over k) and Th = omega diag(x) d_k, the
    predictor-corrector is A + tau/2 (Th A + A Th) + tau^2/2 Th A Th."""
    x, k = ho2d.axes(nx, x_lo, hx, nk, k_lo, hk)
    n = nx * nk
    A = np.zeros((n, n))
    eye = np.eye(nx)
    for i, kv in enumerate(k):
        cols = ho2d.advect(eye, x, np.full(nx, kv), hx, M, g, tau, inflow=inflow)   # row j: image of e_j
        A[i * nx:(i + 1) * nx, i * nx:(i + 1) * nx] = cols.T
    D = ho2d.dk_spectral(np.eye(nk), hk)
    Th = omega * np.kron(D, np.diag(x))
    return A + 0.5 * tau * (Th @ A + A @ Th) + 0.5 * tau * tau * (Th @ A @ Th), x


def test_extrapolated_inflow_admits_a_growing_boundary_mode_zero_inflow_does_not():
    """Spectrum of the one-step operator on the paper's x-line (241 nodes on [-12, 12],
    4 patches of 60 cells, n_nb = 20) and step (tau = 2e-5), k on [-6.4, 6.4) with
    N_k = 8 (the paper's k-box, coarse enough for a dense eigensolve).  Ghost-
    extrapolated inflow has a complex pair of growing modes (rate log|lambda|/tau of
    about 0.59 per unit time, rising with N_k: 0.98 at 16, 1.61 at 32) peaked at the
    x = +-12 boundary columns; with zero inflow every eigenvalue has |lambda| <= 1 to
    rounding.  Both schemes share the periodic spectral k-derivative, so the growth
    comes from the extrapolating inflow closure."""
    rates = {}
    for inflow in ("extrapolate", "zero"):
        L, x = _one_step_matrix(241, -12.0, 0.1, 8, -6.4, 1.6, 60, 20, W, 2e-5, inflow)
        lam, V = np.linalg.eig(L)
        r = np.log(np.abs(lam)) / 2e-5
        top = int(np.argmax(r))
        rates[inflow] = r[top]
        if inflow == "extrapolate":
            amp = np.abs(V[:, top]).reshape(8, 241).max(axis=0)
            assert abs(abs(x[int(np.argmax(amp))]) - 12.0) < 1e-9     # peaked at a boundary column
            assert np.sum(np.isclose(r, r[top], rtol=1e-6)) == 2       # a complex-conjugate pair
    assert 0.5 < rates["extrapolate"] < 0.7
    assert rates["zero"] < 1e-8
