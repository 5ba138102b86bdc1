"""Per-solve QP vectors of a condensed MPC problem. TEST INFRASTRUCTURE ONLY.

Algorithm 1's online stage starts by updating the problem data with the new initial condition.
For the condensed MPC of Sec. IV the cost vector and the bounds are affine in the initial state:
q = F x0 (the paper's g-bar = S'HM x0) and l = lo - E x0, u = hi - E x0 (the paper's c-bar and
d-bar = c, d - G M x0). Written out element by element so that it shares nothing with a BLAS
call elsewhere.
"""

from __future__ import annotations

import numpy as np


def qp_vectors(F, E, lo, hi, x0):
    F = np.asarray(F, float)
    E = np.asarray(E, float)
    x0 = np.asarray(x0, float)
    n, nx = F.shape
    m = E.shape[0]
    q = np.zeros(n)
    s = np.zeros(m)
    for j in range(nx):
        q += F[:, j] * x0[j]
        s += E[:, j] * x0[j]
    return q, np.asarray(lo, float) - s, np.asarray(hi, float) - s
