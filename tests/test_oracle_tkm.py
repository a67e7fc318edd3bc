"""Pins of the truncated-kernel oracle (``oracle/tkm.py``, Sec. 4) against values fixed
by the paper and by mathematics, not by the oracle itself:

* Table 1 (Example 4.1), printed errors for N_k = 8 .. 80 (golden file);
* the Dawson closed form of eq. 4.13 and its twisted extension (the untruncated
  operator of eq. 2.4 on a Gaussian, by completing the square), which fixes the
  modulation signs, the 2/(c_{3,1} i) prefactor and the I+ - I- combination;
* the printed small-|xi| expansion of Uhat_D and its defining radial integral;
* c_{3,1} = 2 pi^2; T real and symmetric in each direction (Sec. 4.1);
* the direct convolution sum of eq. 4.8 equal to the threefold-padded transforms of
  eq. 4.6 (a finite-sum identity: an index or normalisation slip in either fails);
* odd symmetries: Theta flips sign with x~ -> -x~, and is odd in k for f even in k on
  a grid symmetric about 0; Theta = 0 at x = x_A.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

from oracle import tkm

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_tkm.json")


def test_riesz_constant():
    assert abs(tkm.C31 - 2 * math.pi ** 2) < 1e-13


@pytest.mark.parametrize("D", [1.0, 5.5, 27.7])
def test_uhat_small_xi_expansion_and_defining_integral(D):
    # printed expansion: 4 D pi - (2/9) D^3 pi |xi|^2 + O(|xi|^4)
    for xi in (1e-4 / D, 1e-3 / D, 1e-2 / D):
        approx = 4 * D * math.pi - (2.0 / 9.0) * D ** 3 * math.pi * xi ** 2
        got = float(tkm.uhat_D(np.array([xi]), D)[0])
        assert abs(got - approx) <= 0.05 * math.pi * D ** 5 * xi ** 4 + 1e-13 * got
    # defining integral 4 pi int_0^D k^2 |k|^-2 sin(k xi)/(k xi) dk
    for xi in (0.3, 1.7, 6.0):
        ref = 4 * math.pi * integrate.quad(lambda k: math.sin(k * xi) / (k * xi), 0, D, limit=200)[0]
        assert abs(float(tkm.uhat_D(np.array([xi]), D)[0]) - ref) < 1e-10 * abs(ref) + 1e-12
    assert float(tkm.uhat_D(np.array([0.0]), D)[0]) == pytest.approx(4 * math.pi * D, rel=1e-15)


@pytest.mark.parametrize("nk,hk", [((8, 8, 8), (0.5, 0.5, 0.5)), ((6, 8, 4), (0.4, 0.3, 0.7))])
def test_tensor_real_and_symmetric(nk, hk):
    T = tkm.tkm_tensor(nk, hk)
    assert T.shape == (2 * nk[2] - 1, 2 * nk[1] - 1, 2 * nk[0] - 1)
    assert np.max(np.abs(T - T[::-1, :, :])) < 1e-13 * np.max(np.abs(T))
    assert np.max(np.abs(T - T[:, ::-1, :])) < 1e-13 * np.max(np.abs(T))
    assert np.max(np.abs(T - T[:, :, ::-1])) < 1e-13 * np.max(np.abs(T))


@pytest.mark.parametrize("nk,hk", [((8, 8, 8), (0.5, 0.5, 0.5)), ((6, 4, 8), (0.4, 0.9, 0.3))])
def test_direct_sum_equals_threefold_transforms(nk, hk):
    rng = np.random.default_rng(3)
    g = rng.standard_normal(nk[::-1]) + 1j * rng.standard_normal(nk[::-1])
    a = tkm.convolve(g, tkm.tkm_tensor(nk, hk))
    b = tkm.convolve_fft3(g, hk)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def _gaussian_phi(nk, L, alpha, direct=False):
    hk = 2 * L / nk
    k = -L + hk * np.arange(nk)
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    f = np.exp(-(alpha * kk) ** 2)
    if direct:
        phi = tkm.convolve(f, tkm.tkm_tensor((nk,) * 3, (hk,) * 3)).real
    else:
        phi = tkm.convolve_fft3(f, (hk,) * 3).real
    ex = tkm.dawson_phi((alpha * kk) ** 2).real / alpha
    err = phi - ex
    return float(np.max(np.abs(err))), float(np.sqrt(np.sum(err ** 2) * hk ** 3))


def test_table1_errors_reproduced():
    gold = json.load(open(GOLD))
    for row in gold["rows"]:
        linf, l2 = _gaussian_phi(row["nk"], gold["L"], gold["alpha"])
        assert linf == pytest.approx(row["linf"], rel=0.01), row
        assert l2 == pytest.approx(row["l2"], rel=0.01), row


def test_table1_small_rows_by_direct_sum():
    gold = json.load(open(GOLD))
    for row in gold["rows"][:2]:
        linf, l2 = _gaussian_phi(row["nk"], gold["L"], gold["alpha"], direct=True)
        assert linf == pytest.approx(row["linf"], rel=0.01)
        assert l2 == pytest.approx(row["l2"], rel=0.01)


def test_dawson_closed_form_is_the_convolution():
    # eq. 4.13 itself: a radial quadrature of |k|^-2 * e^{-|k|^2} at a few |k|
    for kabs in (0.0, 0.4, 1.3, 3.0):
        def integrand(r, c):
            # angular integral of 1/|k - r e|^2 over the sphere, times e^{-r^2} r^2
            if kabs == 0:
                return 4 * math.pi * math.exp(-r * r)
            return 2 * math.pi * r * math.exp(-r * r) / kabs * math.log(abs((r + kabs) / (r - kabs)))
        ref = integrate.quad(integrand, 0, 12, args=(0,), points=[kabs] if kabs else None, limit=400)[0]
        got = float(tkm.dawson_phi(np.array([kabs ** 2])).real[0])
        assert abs(got - ref) < 1e-8 * ref


@pytest.mark.parametrize("xt,k0", [((0.5, -0.3, 0.2), (0.0, 0.0, 0.0)), ((-0.4, 0.25, 0.6), (0.3, -0.5, 0.2))])
def test_theta_matches_twisted_closed_form(xt, k0):
    nk, L = 32, 6.0
    hk = 2 * L / nk
    k = -L + hk * np.arange(nk)
    f = np.exp(-((k[None, None, :] - k0[0]) ** 2 + (k[None, :, None] - k0[1]) ** 2 + (k[:, None, None] - k0[2]) ** 2))
    th = tkm.theta_point(f, xt, (-L,) * 3, (hk,) * 3)
    ex = tkm.theta_gaussian_exact((k[None, None, :], k[None, :, None], k[:, None, None]), xt, k0)
    assert np.max(np.abs(ex)) > 0.05
    assert np.max(np.abs(th - ex)) < 1e-6 * np.max(np.abs(ex))


def test_theta_symmetries():
    nk, hk = 8, 0.6
    lo = -hk * (nk - 1) / 2                      # symmetric about k = 0
    k = lo + hk * np.arange(nk)
    rng = np.random.default_rng(9)
    # f even in k: symmetrise a random array
    a = rng.standard_normal((nk, nk, nk))
    f = a + a[::-1, ::-1, ::-1]
    T = tkm.tkm_tensor((nk,) * 3, (hk,) * 3)
    xt = (0.7, -0.2, 0.45)
    th = tkm.theta_point(f, xt, (lo,) * 3, (hk,) * 3, T)
    th_neg = tkm.theta_point(f, tuple(-v for v in xt), (lo,) * 3, (hk,) * 3, T)
    s = np.max(np.abs(th))
    assert s > 0
    assert np.max(np.abs(th + th_neg)) < 1e-13 * s
    assert np.max(np.abs(th + th[::-1, ::-1, ::-1])) < 1e-13 * s
    assert np.max(np.abs(tkm.theta_point(a, (0.0, 0.0, 0.0), (lo,) * 3, (hk,) * 3, T))) < 1e-13 * np.max(np.abs(a))
    # the direct-sum and transform routes agree on Theta itself
    th_fft = tkm.theta_point(f, xt, (lo,) * 3, (hk,) * 3)
    assert np.max(np.abs(th - th_fft)) < 1e-12 * s
