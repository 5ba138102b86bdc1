"""Modified Ruiz equilibration of the QP, in FP64. TEST INFRASTRUCTURE ONLY.

Algorithm 1 starts its offline stage by scaling the problem; Sec. III-D (preconditioning) says
the scaling is a modified Ruiz equilibration that, like OSQP's, scales both the KKT matrix and
the cost. Written here from OSQP's published description (Stellato et al. 2020, Sec. 5.1):

KKT matrix M = [[P, A'], [A, 0]]. Each pass:
  1. delta_k = 1 / sqrt(||M[:, k]||_inf) for every column k of the current M (1 for a zero
     column), clipped to [1e-4, 1e4];
  2. P <- Dd P Dd, q <- Dd q, A <- De A Dd, with Dd = diag(delta[:n]), De = diag(delta[n:]);
  3. gamma = 1 / max(mean_j ||P[:, j]||_inf, ||q||_inf) (clipped likewise; 1 if that is 0);
     P <- gamma P, q <- gamma q.
D, E, c accumulate the products of Dd, De and gamma. The scaled problem is
  Pb = c D P D, qb = c D q, Ab = E A D, lb = E l, ub = E u,
with x = D xb, z = zb / E, y = E yb / c (the same QP after a change of variables and of the
constraint rows' units, the cost multiplied by c). Termination is judged on the original
problem's residuals at the unscaled iterates.

Readings: the clipping bounds and the zero-column rule are OSQP's published safeguards; the cost
scale uses the q given at setup, and later q (updates) are scaled with the same c and D.
"""

from __future__ import annotations

import numpy as np

from . import admm

_LO, _HI = 1e-4, 1e4


def _clip_inv_sqrt(v):
    v = np.asarray(v, np.float64)
    d = np.ones_like(v)
    nz = v > 0.0
    d[nz] = 1.0 / np.sqrt(v[nz])
    return np.clip(d, _LO, _HI)


def ruiz(P, q, A, iters: int, cost: bool = True):
    """Returns (D, E, c) after ``iters`` passes."""
    P = np.array(P, np.float64)
    q = np.array(q, np.float64)
    A = np.array(A, np.float64)
    n, m = P.shape[0], A.shape[0]
    D, E, c = np.ones(n), np.ones(m), 1.0
    for _ in range(iters):
        colx = np.maximum(np.max(np.abs(P), axis=0), np.max(np.abs(A), axis=0) if m else 0.0)
        colz = np.max(np.abs(A), axis=1)
        dd, de = _clip_inv_sqrt(colx), _clip_inv_sqrt(colz)
        P = dd[:, None] * P * dd[None, :]
        q = dd * q
        A = de[:, None] * A * dd[None, :]
        D, E = D * dd, E * de
        if cost:
            scale = max(float(np.mean(np.max(np.abs(P), axis=0))), float(np.max(np.abs(q))) if n else 0.0)
            g = 1.0 if scale == 0.0 else float(np.clip(1.0 / scale, _LO, _HI))
            P, q, c = g * P, g * q, c * g
    return D, E, c


def scale_problem(P, q, A, l, u, D, E, c):
    P = np.asarray(P, np.float64)
    A = np.asarray(A, np.float64)
    return (c * (D[:, None] * P * D[None, :]), c * D * np.asarray(q, np.float64), E[:, None] * A * D[None, :],
            E * np.asarray(l, np.float64), E * np.asarray(u, np.float64))


def solve_scaled(P, q, A, l, u, s: admm.Settings, iters: int, *, scaling=None, warm=None, **kw):
    """Scale (Ruiz with ``iters`` passes, or the given (D, E, c)), solve, unscale. ``warm`` is
    in original units. Returns the oracle Result with x, z, y in original units."""
    D, E, c = scaling if scaling is not None else ruiz(P, q, A, iters)
    Pb, qb, Ab, lb, ub = scale_problem(P, q, A, l, u, D, E, c)
    wb = None
    if warm is not None:
        wb = (np.asarray(warm[0]) / D, c * np.asarray(warm[1]) / E, warm[2])
    r = admm.solve(Pb, qb, Ab, lb, ub, s, warm=wb,
                   original=(np.asarray(P, np.float64), np.asarray(q, np.float64), np.asarray(A, np.float64), D, E, c),
                   **kw)
    r.x, r.z, r.y = D * r.x, r.z / E, E * r.y / c
    return r
