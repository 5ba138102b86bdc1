"""Exact solution of a tiny strictly convex QP by active-set enumeration. TEST INFRASTRUCTURE ONLY.

For min 1/2 x'Px + q'x s.t. l <= Ax <= u (paper Sec. II-A, eq. qp_def) with P positive definite
the minimiser is unique. Each row is either at its lower bound, at its upper bound or free
(3^m patterns). For a pattern, the equality-constrained KKT system

    [P  A_S'] [x  ]   [-q ]
    [A_S  0 ] [y_S] = [b_S]

gives a candidate; the optimum is the candidate that is primal feasible and whose multipliers
have the right sign (y_i >= 0 at an upper bound, y_i <= 0 at a lower bound, y_i = 0 if free).
Sign convention: P x + q + A'y = 0 at the optimum, the same as the ADMM dual.
"""

from __future__ import annotations

import itertools

import numpy as np


def solve_qp_enumerate(P, q, A, l, u, tol=1e-9):
    P = np.asarray(P, float)
    q = np.asarray(q, float)
    A = np.asarray(A, float)
    l = np.asarray(l, float)
    u = np.asarray(u, float)
    n, m = P.shape[0], A.shape[0]
    choices = []
    for i in range(m):
        c = [0]  # free
        if np.isfinite(l[i]):
            c.append(-1)  # at lower bound
        if np.isfinite(u[i]) and not (np.isfinite(l[i]) and l[i] == u[i]):
            c.append(1)  # at upper bound (an equality row is handled as "at lower")
        choices.append(c)
    best = None
    for pat in itertools.product(*choices):
        S = [i for i in range(m) if pat[i] != 0]
        k = len(S)
        if k > n:
            continue
        AS = A[S]
        b = np.array([l[i] if pat[i] == -1 else u[i] for i in S])
        K = np.zeros((n + k, n + k))
        K[:n, :n] = P
        K[:n, n:] = AS.T
        K[n:, :n] = AS
        rhs = np.concatenate([-q, b])
        try:
            sol = np.linalg.solve(K, rhs)
        except np.linalg.LinAlgError:
            continue
        if np.linalg.cond(K) > 1e12:
            continue
        x = sol[:n]
        y = np.zeros(m)
        y[S] = sol[n:]
        Ax = A @ x
        scale = 1.0 + np.max(np.abs(Ax))
        if np.any(Ax < l - tol * scale) or np.any(Ax > u + tol * scale):
            continue
        ok = True
        for i in S:
            if l[i] == u[i]:
                continue
            if pat[i] == 1 and y[i] < -tol:
                ok = False
            if pat[i] == -1 and y[i] > tol:
                ok = False
        if not ok:
            continue
        obj = 0.5 * x @ P @ x + q @ x
        if best is None or obj < best[0] - 1e-12:
            best = (obj, x, y)
    if best is None:
        raise ValueError("no feasible active set found (infeasible QP?)")
    return best[1], best[2]
