"""Finite-horizon LQR by the backward Riccati recursion. TEST INFRASTRUCTURE ONLY.

Without inequality constraints the linear MPC problem of eq. mpc_def is an LQR problem solved
exactly by a Riccati recursion (paper Sec. II-C). This is the pin for the condensed QPs that
``workloads.mpc`` builds: their unconstrained minimiser, mapped back through y = S du + M x0,
must equal this rollout.

    X_N = Q_N;  K_k = (R + B'X_{k+1}B)^-1 B'X_{k+1}A;  X_k = Q + A'X_{k+1}(A - B K_k)
    u_k = -K_k x_k,  x_{k+1} = A x_k + B u_k
"""

from __future__ import annotations

import numpy as np


def riccati_rollout(A, B, Q, R, QN, N, x0):
    X = QN.copy()
    gains = [None] * N
    for k in range(N - 1, -1, -1):
        Kk = np.linalg.solve(R + B.T @ X @ B, B.T @ X @ A)
        gains[k] = Kk
        X = Q + A.T @ X @ (A - B @ Kk)
        X = 0.5 * (X + X.T)
    xs = [np.asarray(x0, float)]
    us = []
    for k in range(N):
        uk = -gains[k] @ xs[-1]
        us.append(uk)
        xs.append(A @ xs[-1] + B @ uk)
    return np.array(us), np.array(xs[1:])


def dare_residual(A, B, Q, R, K):
    """Residual of the stationary Riccati equation at the gain K (zero for the LQR gain)."""
    # X solves X = Q + K'RK + (A-BK)'X(A-BK) for the closed loop; then K must equal
    # (R + B'XB)^-1 B'XA.
    n = A.shape[0]
    Ac = A - B @ K
    lhs = np.eye(n * n) - np.kron(Ac.T, Ac.T)
    X = np.linalg.solve(lhs, (Q + K.T @ R @ K).reshape(-1)).reshape(n, n)
    K2 = np.linalg.solve(R + B.T @ X @ B, B.T @ X @ A)
    return float(np.max(np.abs(K2 - K)))
