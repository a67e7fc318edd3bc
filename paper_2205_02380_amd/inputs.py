"""Seeded synthetic inputs for the CHASM advection step.

This module is the only code shared between the HIP path and the FP64 oracle.  It
holds the workload definitions and the seeded generators of initial data: Gaussian
Wigner packets (the paper's initial states are Gaussian coherent states, Sec. 5.1 and
5.3-5.4), polynomial fields and the serving request trace.  It contains none of the
advection method's arithmetic.  All randomness comes from numpy's PCG64
(``numpy.random.default_rng(seed)``).

Layout of a field: ``f[b][k3][k2][k1][x3][x2][x1]``, x1 fastest.  Axis d has nodes
``x_lo[d] + i*h[d]``, ``h[d] = (x_hi[d]-x_lo[d])/nx[d]`` (half-open extents), and
likewise for k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Sequence, Tuple

import numpy as np

PI3 = math.pi ** -3


@dataclass(frozen=True)
class Grid:
    nx: Tuple[int, int, int]
    x_lo: Tuple[float, float, float]
    x_hi: Tuple[float, float, float]
    nk: Tuple[int, int, int]
    k_lo: Tuple[float, float, float]
    k_hi: Tuple[float, float, float]

    @property
    def hx(self) -> Tuple[float, float, float]:
        return tuple((self.x_hi[d] - self.x_lo[d]) / self.nx[d] for d in range(3))

    @property
    def hk(self) -> Tuple[float, float, float]:
        return tuple((self.k_hi[d] - self.k_lo[d]) / self.nk[d] for d in range(3))

    def x_axis(self, d: int) -> np.ndarray:
        return self.x_lo[d] + np.arange(self.nx[d], dtype=np.float64) * self.hx[d]

    def k_axis(self, d: int) -> np.ndarray:
        return self.k_lo[d] + np.arange(self.nk[d], dtype=np.float64) * self.hk[d]

    @property
    def cube(self) -> int:
        return self.nx[0] * self.nx[1] * self.nx[2]

    @property
    def nkpts(self) -> int:
        return self.nk[0] * self.nk[1] * self.nk[2]

    @property
    def points(self) -> int:
        return self.cube * self.nkpts

    def shape(self, nbatch: int = 1) -> Tuple[int, ...]:
        s = (self.nk[2], self.nk[1], self.nk[0], self.nx[2], self.nx[1], self.nx[0])
        return ((nbatch,) + s) if nbatch > 1 else s


def cubic_grid(n: int, xr: float, nk: int, kr: float) -> Grid:
    return Grid((n, n, n), (-xr,) * 3, (xr,) * 3, (nk, nk, nk), (-kr,) * 3, (kr,) * 3)


@dataclass(frozen=True)
class Packets:
    """Gaussian Wigner packets f0 = sum_p w_p pi^-3 exp(-|x-c_p|^2/s_p^2 - s_p^2 |k-k0_p|^2)."""
    w: np.ndarray      # (P,)
    c: np.ndarray      # (P, 3)
    k0: np.ndarray     # (P, 3)
    s: np.ndarray      # (P,)

    @property
    def n(self) -> int:
        return int(self.w.shape[0])


def single_packet(c=(-1.0, 0.0, 1.0), k0=(0.5, 0.0, 0.0), s=1.0, w=1.0) -> Packets:
    return Packets(np.array([w], float), np.array([c], float), np.array([k0], float), np.array([s], float))


def random_packets(n: int, seed: int, c_range=(-4.0, 4.0), k0_range=(-1.0, 1.0),
                   s_range=(0.8, 1.5), w_range=(0.5, 1.0)) -> Packets:
    rng = np.random.default_rng(seed)
    c = rng.uniform(c_range[0], c_range[1], size=(n, 3))
    k0 = rng.uniform(k0_range[0], k0_range[1], size=(n, 3))
    s = rng.uniform(s_range[0], s_range[1], size=n)
    w = rng.uniform(w_range[0], w_range[1], size=n)
    return Packets(w, c, k0, s)


def packet_factors(grid: Grid, pk: Packets):
    """Per-packet separable factors: coef[p] and, per axis d, gx[p][d] (nx_d,) and
    gk[p][d] (nk_d,), so that f0 = sum_p coef[p] prod_d gx[p][d](x_d) gk[p][d](k_d)."""
    coef = pk.w * PI3
    gx = [[np.exp(-((grid.x_axis(d) - pk.c[p, d]) / pk.s[p]) ** 2) for d in range(3)] for p in range(pk.n)]
    gk = [[np.exp(-(pk.s[p] * (grid.k_axis(d) - pk.k0[p, d])) ** 2) for d in range(3)] for p in range(pk.n)]
    return coef, gx, gk


def fill_separable(out, coef, ux, uk=None):
    """Write sum_p coef[p] prod_d U[p][d][k_d, x_d] into ``out`` (a torch tensor of shape
    [k3][k2][k1][x3][x2][x1], any dtype/device), one k3-slab at a time in FP64.

    ux[p][d] is either (nx_d,) (no k dependence, then uk[p][d] (nk_d,) multiplies)
    or (nk_d, nx_d)."""
    import torch
    dev = out.device
    nk3, nk2, nk1, n3, n2, n1 = out.shape

    def as2d(p, d, nk):
        u = torch.as_tensor(np.asarray(ux[p][d]), dtype=torch.float64, device=dev)
        if u.dim() == 1:
            kf = torch.as_tensor(np.asarray(uk[p][d]), dtype=torch.float64, device=dev)
            u = kf[:, None] * u[None, :]
        return u

    U = [[as2d(p, d, (nk1, nk2, nk3)[d]) for d in range(3)] for p in range(len(coef))]
    for i3 in range(nk3):
        acc = None
        for p in range(len(coef)):
            a1, a2, a3 = U[p][0], U[p][1], U[p][2][i3]          # (nk1,n1), (nk2,n2), (n3,)
            t = a2[:, None, :, None] * a1[None, :, None, :]      # [k2][k1][x2][x1]
            t = t[:, :, None, :, :] * a3[None, None, :, None, None] * float(coef[p])
            acc = t if acc is None else acc + t
        out[i3].copy_(acc.to(out.dtype))
    return out


def gaussian_field(grid: Grid, pk: Packets, dtype=None, device="cpu"):
    """f0 on the grid as a torch tensor, evaluated in FP64 then cast to ``dtype``."""
    import torch
    dtype = dtype or torch.float64
    out = torch.empty(grid.shape(), dtype=dtype, device=device)
    coef, gx, gk = packet_factors(grid, pk)
    return fill_separable(out, coef, gx, gk)


# ---------------------------------------------------------------------------
# Cubic polynomials in x (total degree <= 3): 20 monomials x1^a x2^b x3^c.
MONOMIALS: List[Tuple[int, int, int]] = [
    (a, b, c) for t in range(4) for c in range(t + 1) for b in range(t + 1 - c) for a in [t - b - c]
]


def cubic_coeffs(seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(len(MONOMIALS))


def cubic_eval(coeffs, x1, x2, x3):
    """p(x) = sum_m coeffs[m] x1^a x2^b x3^c; arrays broadcast (numpy or torch)."""
    acc = 0.0
    for cf, (a, b, c) in zip(coeffs, MONOMIALS):
        acc = acc + float(cf) * (x1 ** a) * (x2 ** b) * (x3 ** c)
    return acc


# ---------------------------------------------------------------------------
# Workloads.
@dataclass(frozen=True)
class Workload:
    name: str
    grid: Grid
    patch: Tuple[int, int, int]
    ghost: int
    dt: float
    steps: int
    packets: Packets
    dtype: str = "f32"

    def describe(self) -> dict:
        g = self.grid
        return {
            "workload": self.name,
            "nx": list(g.nx), "nk": list(g.nk),
            "x": [g.x_lo[0], g.x_hi[0]], "k": [g.k_lo[0], g.k_hi[0]],
            "patch": list(self.patch), "ghost": self.ghost, "dt": self.dt, "steps": self.steps,
            "packets": self.packets.n, "points": g.points,
        }


def workload(name: str) -> Workload:
    """The seeded workloads: 'C1' .. 'C4' (one job each)."""
    if name == "C1":
        return Workload("C1 fp64 16^3x8^3", cubic_grid(16, 8.0, 8, 2.0), (8, 8, 8), 4, 0.05, 10,
                        single_packet(), "f64")
    if name == "C2":
        return Workload("C2 fp32 32^3x16^3", cubic_grid(32, 12.0, 16, 4.0), (8, 8, 8), 6, 0.02, 100,
                        random_packets(4, 2))
    if name == "C3":
        return Workload("C3 fp32 48^3x24^3", cubic_grid(48, 16.0, 24, 4.0), (16, 16, 16), 8, 0.02, 50,
                        random_packets(4, 3))
    if name == "C4":
        return Workload("C4 fp32 64^3x32^3", cubic_grid(64, 16.0, 32, 4.0), (16, 16, 16), 8, 0.02, 50,
                        random_packets(8, 4, s_range=(0.6, 1.2)))
    raise KeyError(name)


def k_sample(grid: Grid, fraction: float, seed: int) -> np.ndarray:
    """Seeded sample of k-points as (i1, i2, i3) rows, without replacement."""
    n = grid.nkpts
    m = max(1, int(round(fraction * n)))
    idx = np.sort(np.random.default_rng(seed).choice(n, size=m, replace=False))
    i1 = idx % grid.nk[0]
    i2 = (idx // grid.nk[0]) % grid.nk[1]
    i3 = idx // (grid.nk[0] * grid.nk[1])
    return np.stack([i1, i2, i3], axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# Serving trace: Poisson arrivals of advection requests of mixed shapes.
SERVING_SHAPES: List[Grid] = [
    cubic_grid(16, 8.0, 8, 2.0),
    cubic_grid(24, 12.0, 12, 3.0),
    cubic_grid(32, 12.0, 16, 4.0),
    Grid((48, 48, 48), (-16.0,) * 3, (16.0,) * 3, (16, 16, 16), (-4.0,) * 3, (4.0,) * 3),
]


@dataclass(frozen=True)
class Request:
    rid: int
    arrival: float
    grid: Grid
    steps: int
    dt: float
    packets: Packets
    patch: Tuple[int, int, int] = (8, 8, 8)
    ghost: int = 6


def serving_trace(n: int = 200, rate: float = 20.0, seed: int = 5,
                  shapes: Sequence[Grid] = SERVING_SHAPES, steps_range=(10, 200),
                  dts=(0.01, 0.02, 0.05)) -> List[Request]:
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    shape_i = rng.integers(0, len(shapes), size=n)
    steps = rng.integers(steps_range[0], steps_range[1] + 1, size=n)
    dt_i = rng.integers(0, len(dts), size=n)
    return [Request(i, float(t[i]), shapes[int(shape_i[i])], int(steps[i]), float(dts[int(dt_i[i])]),
                    random_packets(4, 5000 + i)) for i in range(n)]


def gaussian_cubes(grid: Grid, pk: Packets, kidx) -> np.ndarray:
    """FP64 x-cubes of f0 at the k-points kidx[n] = (i1, i2, i3): array [n][x3][x2][x1]."""
    coef, gx, gk = packet_factors(grid, pk)
    kidx = np.asarray(kidx).reshape(-1, 3)
    out = np.zeros((kidx.shape[0], grid.nx[2], grid.nx[1], grid.nx[0]))
    for p in range(pk.n):
        cube = gx[p][2][:, None, None] * gx[p][1][None, :, None] * gx[p][0][None, None, :]
        for n, (i1, i2, i3) in enumerate(kidx):
            out[n] += coef[p] * gk[p][0][i1] * gk[p][1][i2] * gk[p][2][i3] * cube
    return out
