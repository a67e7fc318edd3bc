"""FP64 oracle of the visualisation observables of Sec. 5: the reduced Wigner functions
W_j(x_j, k_j) (f integrated over the other two x and the other two k variables) and
the spatial marginal P(x1, x2) (f integrated over x3 and k).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it; it shares no code with the HIP
library.  Integrals are cell sums times the spacings of the integrated variables (the
paper replaces integrals by grid averages, Sec. 5).  Pinned in
``tests/test_oracle_observables.py`` by the closed-form marginals of a Gaussian packet
and by the mass identity.
"""
from __future__ import annotations

import numpy as np


def marginals(f: np.ndarray, hx, hk):
    """f is [k3][k2][k1][x3][x2][x1] (or with a leading batch axis).  Returns
    (W1 [k1][x1], W2 [k2][x2], W3 [k3][x3], P [x2][x1]), with the batch axis first when
    f has one."""
    f = np.asarray(f, dtype=np.float64)
    lead = f.ndim - 6
    ax = lambda *a: tuple(lead + i for i in a)        # axes counted from the 6-D part
    v = [hx[d] * hk[d] for d in range(3)]
    w1 = f.sum(axis=ax(0, 1, 3, 4)) * (v[1] * v[2])     # keep k1 (2), x1 (5)
    w2 = f.sum(axis=ax(0, 2, 3, 5)) * (v[0] * v[2])     # keep k2 (1), x2 (4)
    w3 = f.sum(axis=ax(1, 2, 4, 5)) * (v[0] * v[1])     # keep k3 (0), x3 (3)
    p = f.sum(axis=ax(0, 1, 2, 3)) * (hx[2] * hk[0] * hk[1] * hk[2])   # keep x2, x1
    return w1, w2, w3, p
