"""FP64 CPU oracle for the truncated-kernel evaluation of the Coulomb pseudo-differential
operator Theta_V (Sec. 4).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP
library; numpy's FFT and scipy's sine integral / Dawson function serve as library
primitives for single steps, nothing else.

What is computed, in the paper's order (atomic units, attractive Coulomb potential
V(x) = -1/|x - x_A|, Sec. 2.1):

* ``c_coef``        c_{n,alpha} = pi^{n/2} 2^alpha Gamma(alpha/2) / Gamma((n - alpha)/2)
                    (the constant of eq. 2.4; c_{3,1} = 2 pi^2).
* ``uhat_D``        Fourier transform of the kernel |k|^{-2} truncated at |k| <= D:
                    4 pi Si(|xi| D) / |xi|, and 4 pi D at xi = 0 (Sec. 4.1).
* ``tkm_tensor``    the convolution tensor T_p of eq. 4.9 over the dual index set of
                    eq. 4.10 (threefold grid, xi_n = 2 pi n / (3 N_k hk)), for
                    |p_d| <= N_k - 1, by one inverse DFT of size (3 N_k)^3.
* ``convolve``      Phi_p = sum_{p'} T_{p-p'} g_{p'} (eq. 4.8), the plain double sum.
* ``convolve_fft3`` the same Phi from eq. 4.6 as printed: zero-pad g threefold, DFT,
                    multiply by Uhat_D(xi_n), inverse DFT, keep the original points.
* ``theta_point``   Theta_V^T[f](x, k_p) of eq. 4.6 at one x: both twisted terms,
                    e^{2i x~.k} F^{-1}[Uhat_D F(e^{-2i x~.k} f)] and its mirror, times
                    2/(c_{3,1} i), with x~ = x - x_A.
* ``theta6d``       ``theta_point`` at every sampled x of a 6-D field.

Readings (the paper leaves these implicit): the k grid is half-open, k_i = k_lo + i hk
with N_k (even) nodes per axis; Omega is the box of side N_k hk, so D = |(N_k hk)_d|
(its diameter).  For a grid that is not cubic the dual spacing is per axis.
Pinned in ``tests/test_oracle_tkm.py`` against Table 1 (Example 4.1), the Dawson closed
form (eq. 4.13) and its twisted extension, the printed small-|xi| expansion of
Uhat_D, the defining integral of Uhat_D, the symmetry of T, and the equality of the two
routes above.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np
from scipy import special


def c_coef(n: int, alpha: float) -> float:
    """c_{n,alpha} of the Riesz-kernel constant (Sec. 2.1)."""
    return math.pi ** (n / 2) * 2.0 ** alpha * math.gamma(alpha / 2) / math.gamma((n - alpha) / 2)


C31 = c_coef(3, 1)


def box_diameter(nk: Sequence[int], hk: Sequence[float]) -> float:
    """D = diam Omega for the box of side nk_d * hk_d (Sec. 4.1)."""
    return math.sqrt(sum((n * h) ** 2 for n, h in zip(nk, hk)))


def uhat_D(r, D: float):
    """4 pi Si(r D) / r, with the limit 4 pi D at r = 0 (Sec. 4.1)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.full(r.shape, 4.0 * math.pi * D)
    nz = r > 0
    out[nz] = 4.0 * math.pi * special.sici(r[nz] * D)[0] / r[nz]
    return out


def _dual_grid(nk: Sequence[int], hk: Sequence[float]):
    """|xi_n| on the (3 nk)^3 dual grid in DFT order, array [n3][n2][n1] (eq. 4.10)."""
    xs = []
    for n, h in zip(nk, hk):
        if n % 2:
            raise ValueError("the dual index set of eq. 4.10 needs an even number of k nodes")
        m = 3 * n
        idx = np.fft.fftfreq(m, d=1.0 / m)          # 0..m/2-1, -m/2..-1: the set of eq. 4.10
        xs.append(2.0 * math.pi * idx / (m * h))
    x1, x2, x3 = xs
    return np.sqrt(x3[:, None, None] ** 2 + x2[None, :, None] ** 2 + x1[None, None, :] ** 2)


def tkm_tensor(nk: Sequence[int], hk: Sequence[float]) -> np.ndarray:
    """T_p of eq. 4.9 for p_d = -(nk_d - 1) .. nk_d - 1, as a real array
    [p3 + nk3 - 1][p2 + nk2 - 1][p1 + nk1 - 1]."""
    D = box_diameter(nk, hk)
    U = uhat_D(_dual_grid(nk, hk), D)
    full = np.fft.ifftn(U)                           # (1/M^3) sum_n U_n e^{+2 pi i p.n / M}
    n1, n2, n3 = nk
    i3 = np.arange(-(n3 - 1), n3) % (3 * n3)
    i2 = np.arange(-(n2 - 1), n2) % (3 * n2)
    i1 = np.arange(-(n1 - 1), n1) % (3 * n1)
    T = full[np.ix_(i3, i2, i1)]
    assert np.max(np.abs(T.imag)) <= 1e-12 * np.max(np.abs(T.real))
    return np.ascontiguousarray(T.real)


def convolve(g: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Phi_p = sum_{p'} T_{p - p'} g_{p'} over the grid (eq. 4.8); g is [k3][k2][k1]."""
    n3, n2, n1 = g.shape
    out = np.zeros(g.shape, dtype=np.result_type(g.dtype, T.dtype))
    for q3 in range(n3):
        for q2 in range(n2):
            for q1 in range(n1):
                out += T[n3 - 1 - q3:2 * n3 - 1 - q3, n2 - 1 - q2:2 * n2 - 1 - q2,
                         n1 - 1 - q1:2 * n1 - 1 - q1] * g[q3, q2, q1]
    return out


def convolve_fft3(g: np.ndarray, hk: Sequence[float]) -> np.ndarray:
    """Phi of eq. 4.6's inner part: threefold zero padding, DFT of size (3 N_k)^3,
    multiplication by Uhat_D(xi_n), inverse DFT, the original N_k^3 points."""
    n3, n2, n1 = g.shape
    nk = (n1, n2, n3)
    U = uhat_D(_dual_grid(nk, hk), box_diameter(nk, hk))
    pad = np.zeros((3 * n3, 3 * n2, 3 * n1), dtype=np.complex128)
    pad[:n3, :n2, :n1] = g
    return np.fft.ifftn(U * np.fft.fftn(pad))[:n3, :n2, :n1]


def k_axes(nk: Sequence[int], k_lo: Sequence[float], hk: Sequence[float]):
    return [k_lo[d] + hk[d] * np.arange(nk[d], dtype=np.float64) for d in range(3)]


def theta_point(fk: np.ndarray, xt: Sequence[float], k_lo: Sequence[float], hk: Sequence[float],
                T: np.ndarray = None) -> np.ndarray:
    """Theta_V^T[f](x, k_p) at one x (eq. 4.6), x~ = xt.  fk is f(x, .) as [k3][k2][k1].
    With T given the convolutions use the direct sum of eq. 4.8, else eq. 4.6's
    threefold-padded transforms."""
    n3, n2, n1 = fk.shape
    k1, k2, k3 = k_axes((n1, n2, n3), k_lo, hk)
    ph = 2.0 * (xt[0] * k1[None, None, :] + xt[1] * k2[None, :, None] + xt[2] * k3[:, None, None])
    conv = (lambda g: convolve(g, T)) if T is not None else (lambda g: convolve_fft3(g, hk))
    pre = 2.0 / (C31 * 1j)
    i_plus = pre * np.exp(1j * ph) * conv(np.exp(-1j * ph) * fk)
    i_minus = pre * np.exp(-1j * ph) * conv(np.exp(1j * ph) * fk)
    th = i_plus - i_minus
    return th.real


def theta6d(f: np.ndarray, x_axes: Sequence[np.ndarray], x_a: Sequence[float], k_lo: Sequence[float],
            hk: Sequence[float], xidx: np.ndarray, direct: bool = False) -> np.ndarray:
    """Theta_V^T at the sampled x-points xidx (rows (i1, i2, i3)) of the field
    f[k3][k2][k1][x3][x2][x1]; returns [n][k3][k2][k1]."""
    nk = (f.shape[2], f.shape[1], f.shape[0])
    T = tkm_tensor(nk, hk) if direct else None
    out = np.empty((len(xidx),) + f.shape[:3])
    for n, (i1, i2, i3) in enumerate(xidx):
        xt = (x_axes[0][i1] - x_a[0], x_axes[1][i2] - x_a[1], x_axes[2][i3] - x_a[2])
        out[n] = theta_point(f[:, :, :, i3, i2, i1], xt, k_lo, hk, T)
    return out


def dawson_phi(z: np.ndarray) -> np.ndarray:
    """Phi(k) = (|k|^{-2} * e^{-|k|^2})(k) = 2 pi^{3/2} D(s)/s with s = |k| (eq. 4.13);
    an even entire function of s, so z may be complex (s^2 = z.z)."""
    s2 = np.asarray(z, dtype=np.complex128)
    s = np.sqrt(s2)
    small = np.abs(s2) < 1e-12
    sd = np.where(small, 1.0, s)
    return np.where(small, 2.0 * math.pi ** 1.5 * (1.0 - 2.0 * s2 / 3.0),
                    2.0 * math.pi ** 1.5 * special.dawsn(sd) / sd)


def theta_gaussian_exact(k_grid: Tuple[np.ndarray, np.ndarray, np.ndarray], xt: Sequence[float],
                         k0: Sequence[float]) -> np.ndarray:
    """Theta_V[f] of the untruncated operator (eq. 2.4) for f(k) = e^{-|k - k0|^2} at
    x~ = xt, on a k grid given as broadcastable (k1, k2, k3) arrays:
    (2/pi^2) Im(e^{2i x~.(k - k0) - |x~|^2} Phi(k - k0 + i x~)), which follows from
    eq. 4.2 by completing the square in the twisted Gaussian."""
    q = [k_grid[d] - k0[d] for d in range(3)]
    z2 = sum((q[d] + 1j * xt[d]) ** 2 for d in range(3))
    twist = np.exp(2j * sum(xt[d] * q[d] for d in range(3)) - sum(x * x for x in xt))
    return (4.0 / C31) * np.imag(twist * dawson_phi(z2))
