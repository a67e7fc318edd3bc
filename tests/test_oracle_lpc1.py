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


# ---- temporal order of the predictor-corrector structure (Sec. 2.2) ---------------
# With exact linear operators in place of the characteristic step and Theta -- the flow
# A = e^{tau D} of a linear "transport" generator D and a fixed matrix T for Theta --
# the exact solution of f' = (D + T) f is e^{t (D + T)} f0.  LPC1 is second order:
# at fixed end time the error falls ~4x per halving of tau.  D and T do not commute,
# so a structural slip that keeps first-order consistency (a corrector that reuses
# Theta[f^n] o A_tau for Theta[f~], a predictor without its tau term) falls only ~2x.
from scipy.linalg import expm


def _linear_system(n=12, seed=7):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((n, n))
    D = 1.5 * (S - S.T) / np.sqrt(n)          # skew: a norm-preserving flow, like transport
    T = rng.standard_normal((n, n)) / np.sqrt(n)
    f0 = rng.standard_normal(n)
    assert np.linalg.norm(D @ T - T @ D) > 0.5
    return D, T, f0


def _global_errors(step, taus, t_end=1.0):
    D, T, f0 = _linear_system()
    exact = expm(t_end * (D + T)) @ f0
    errs = []
    for tau in taus:
        A_tau = expm(tau * D)
        f = f0.copy()
        for _ in range(int(round(t_end / tau))):
            f = step(f, lambda g: A_tau @ g, lambda g: T @ g, tau)
        errs.append(np.max(np.abs(f - exact)) / np.max(np.abs(exact)))
    return np.array(errs)


TAUS = (1 / 8, 1 / 16, 1 / 32, 1 / 64)


def _ratios(errs):
    return errs[:-1] / errs[1:]


def test_lpc1_step_is_second_order_in_time():
    r = _ratios(_global_errors(lpc1.lpc1_step, TAUS))
    assert np.all((3.5 < r) & (r < 4.5)), r


def _corrector_reuses_theta_of_fn(f, A, Th, tau):
    th = Th(f)
    af = A(f)
    ath = A(th)
    return af + 0.5 * tau * ath + 0.5 * tau * ath


def _predictor_without_tau_term(f, A, Th, tau):
    th = Th(f)
    af = A(f)
    ath = A(th)
    return af + 0.5 * tau * Th(af) + 0.5 * tau * ath


def test_planted_lpc1_slips_fall_at_first_order():
    for bad in (_corrector_reuses_theta_of_fn, _predictor_without_tau_term):
        r = _ratios(_global_errors(bad, TAUS))
        assert np.all((1.7 < r) & (r < 2.4)), (bad.__name__, r)
        assert not np.all((3.5 < r) & (r < 4.5))
