"""FP64 oracle of the LPC1 time step (Sec. 2.2) of the Wigner-Coulomb equation:

  predictor  f~      = f^n o A_tau + tau Theta[f^n] o A_tau
  corrector  f^{n+1} = f^n o A_tau + tau/2 Theta[f~] + tau/2 Theta[f^n] o A_tau,

with g o A_tau the characteristic step of the advection oracle (``oracle.advect6d``,
Sec. 3) and Theta the truncated-kernel operator of the TKM oracle (``oracle.tkm``,
Sec. 4) summed over the nuclei.

TEST INFRASTRUCTURE, NOT PRODUCT CODE; it shares no code with the HIP library.  Pinned
in ``tests/test_oracle_lpc1.py``: with no nuclei (Theta = 0) a step is exactly the
characteristic step; as tau -> 0, (step - characteristic step)/tau tends to Theta[f]
at first order in tau (which fixes the tau and tau/2 coefficients); the step is linear;
and ``lpc1_step`` with exact linear operators in place of A_tau and Theta (the flow of
a linear system, where e^{tau(D + T)} is the exact solution) converges at second order
in tau, which a corrector that reuses Theta[f^n] o A_tau for Theta[f~], or a predictor
without its tau term, does not.  The component operators carry their own pins.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import tkm


def theta_field(f, grid, nuclei, charges, direct=True):
    """Theta^T[f] at every x of the field f[k3][k2][k1][x3][x2][x1] (direct sums of
    eq. 4.8, or eq. 4.6's threefold transforms when direct is False)."""
    out = np.zeros_like(f, dtype=np.float64)
    nk = (grid.nk[0], grid.nk[1], grid.nk[2])
    T = tkm.tkm_tensor(nk, grid.hk) if direct else None
    xs = [grid.x_axis(d) for d in range(3)]
    for xa, z in zip(nuclei, charges):
        for i3 in range(grid.nx[2]):
            for i2 in range(grid.nx[1]):
                for i1 in range(grid.nx[0]):
                    xt = (xs[0][i1] - xa[0], xs[1][i2] - xa[1], xs[2][i3] - xa[2])
                    out[:, :, :, i3, i2, i1] += z * tkm.theta_point(f[:, :, :, i3, i2, i1], xt, grid.k_lo, grid.hk, T)
    return out


def advect(f, grid, patch, ghost, tau):
    P = (patch,) * 3 if isinstance(patch, int) else patch
    return oracle.advect6d(f, grid.nx, grid.hx, grid.nk, grid.k_lo, grid.hk, P, ghost, tau, 1)


def lpc1_step(f, A, Th, tau):
    """One LPC1 step (Sec. 2.2) with the characteristic step A(g) = g o A_tau and the
    operator Th(g) = Theta[g] given as callables."""
    th = Th(f)
    af = A(f)
    ath = A(th)
    ft = af + tau * ath                                  # predictor
    return af + 0.5 * tau * Th(ft) + 0.5 * tau * ath     # corrector


def lpc1(f, grid, patch, ghost, tau, nsteps, nuclei, charges, direct=True):
    f = np.asarray(f, dtype=np.float64)
    A = lambda g: advect(g, grid, patch, ghost, tau)
    Th = lambda g: theta_field(g, grid, nuclei, charges, direct)
    for _ in range(nsteps):
        f = lpc1_step(f, A, Th, tau)
    return f
