"""FP64 oracle of the 2-D (x, k) harmonic-oscillator workload of Sec. 5.1.

TEST INFRASTRUCTURE, NOT PRODUCT CODE (used by ``tests/`` and the CPU-baseline leg of
``bench.py`` only; it shares no code with the HIP library).

The Wigner equation with V = omega x^2 / 2 (m = hbar = 1) reads
  d_t f + k d_x f = Theta[f],   Theta[f] = omega x d_k f      (eq. 5.1)
and is advanced by LPC1 (Sec. 2.2): the characteristic step in x of every k-line with
the patched cubic spline of Sec. 3 (the C oracle's line routine, PMBC, natural closure),
and Theta from the spectral derivative in k on the periodic k-grid (numpy's FFT as a
library primitive; the Nyquist mode's derivative is set to zero).  Departure points
outside [x_0, x_{N-1}] give 0 (zero inflow) unless inflow="extrapolate".  The exact solution
is f0 along the reverse-time Hamiltonian flow of eq. 5.2:
  X = cos(sqrt(w) t) x - sin(sqrt(w) t) k / sqrt(w),
  K = sqrt(w) sin(sqrt(w) t) x + cos(sqrt(w) t) k.
Pinned in ``tests/test_oracle_ho2d.py``.
"""
from __future__ import annotations

import math

import numpy as np

import oracle


def axes(nx, x_lo, hx, nk, k_lo, hk):
    return x_lo + hx * np.arange(nx), k_lo + hk * np.arange(nk)


def advect(f, x, k, hx, M, g, tau, stencil=None, inflow="zero"):
    """One characteristic step of every k-line f[k][:] (shift alpha = k tau / hx).
    inflow "zero": nodes whose departure point x_j - alpha hx lies outside
    [x_0, x_{N-1}] get 0; "extrapolate": the outer patch evaluates them with its ghost
    coefficients (as on the 6-D path)."""
    N = f.shape[1]
    c = stencil if stencil is not None else oracle.stencils(N, M, g, hx)
    out = np.empty_like(f)
    j = np.arange(N)
    for i, kv in enumerate(k):
        a = kv * tau / hx
        out[i] = oracle.line(N, M, g, hx, a, f[i], c=c)
        if inflow == "zero":
            t = j - a                               # departure point in units of hx from x_0
            out[i][(t < 0) | (t > N - 1)] = 0.0
    return out


def dk_spectral(f, hk):
    """Spectral derivative along k (axis 0) of f[k][x] on the periodic k-grid."""
    n = f.shape[0]
    xi = 2.0 * math.pi * np.fft.fftfreq(n, d=hk)
    if n % 2 == 0:
        xi[n // 2] = 0.0
    return np.real(np.fft.ifft(1j * xi[:, None] * np.fft.fft(f, axis=0), axis=0))


def theta(f, x, hk, omega):
    return omega * x[None, :] * dk_spectral(f, hk)


def lpc1(f, x, k, hx, hk, M, g, omega, tau, nsteps, inflow="zero"):
    c = oracle.stencils(f.shape[1], M, g, hx)
    f = np.asarray(f, dtype=np.float64)
    for _ in range(nsteps):
        th = theta(f, x, hk, omega)
        af = advect(f, x, k, hx, M, g, tau, c, inflow)
        ath = advect(th, x, k, hx, M, g, tau, c, inflow)
        ft = af + tau * ath
        f = af + 0.5 * tau * theta(ft, x, hk, omega) + 0.5 * tau * ath
    return f


def f0(x, k):
    """The initial packet of Sec. 5.1: pi^-1 exp(-(x - 1)^2 / 2 - 2 k^2)."""
    return np.exp(-0.5 * (x - 1.0) ** 2 - 2.0 * k ** 2) / math.pi


def exact(x, k, t, omega):
    """f0 along the reverse-time Hamiltonian flow (eq. 5.2), on the grid [k][x]."""
    s = math.sqrt(omega)
    X = math.cos(s * t) * x[None, :] - math.sin(s * t) * k[:, None] / s
    K = s * math.sin(s * t) * x[None, :] + math.cos(s * t) * k[:, None]
    return f0(X, K)
