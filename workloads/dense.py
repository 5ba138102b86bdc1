"""Seeded random dense QPs (the paper's first benchmark, Sec. V-A, has n/4 equality and n/4
inequality rows; it does not give the distribution, so the one below is this project's choice).

Recipe for ``random_qp(n, m_eq, m_ineq, seed)``, draws in this order from ``default_rng(seed)``:
  * M ~ N(0,1)^{n x n};  P = M'M / n + reg * I  (strictly convex, reg = 1e-2 by default)
  * q ~ N(0,1)^n
  * A ~ N(0,1)^{m x n} / sqrt(n),  m = m_eq + m_ineq, equality rows first
  * x_f ~ N(0,1)^n, a point that makes the constraints feasible
  * equality rows: l = u = A x_f;  inequality rows: l = A x_f - w, u = A x_f + w, w ~ U[0,1]
"""

from __future__ import annotations

import numpy as np


def random_qp(n: int, m_eq: int, m_ineq: int, seed: int, reg: float = 1e-2):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    P = M.T @ M / n + reg * np.eye(n)
    P = 0.5 * (P + P.T)
    q = rng.standard_normal(n)
    m = m_eq + m_ineq
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    xf = rng.standard_normal(n)
    Ax = A @ xf
    w = rng.uniform(0.0, 1.0, m)
    l = Ax - w
    u = Ax + w
    l[:m_eq] = Ax[:m_eq]
    u[:m_eq] = Ax[:m_eq]
    return P, q, A, l, u


def random_box_qp(n: int, seed: int):
    """Separable QP: P diagonal, A = I, finite box. Its solution is known in closed form."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 2.0, n)
    P = np.diag(d)
    q = rng.standard_normal(n) * 2.0
    A = np.eye(n)
    c = rng.standard_normal(n) * 0.5
    w = rng.uniform(0.1, 1.0, n)
    return P, q, A, c - w, c + w
