"""Random linear MPC problems, condensed into dense QPs (paper Sec. IV, Dense MPC).

The linear MPC problem (paper Sec. II-C, eq. mpc_def) is

    min  sum_{k=0}^{N-1} 1/2 x_k'Q x_k + 1/2 u_k'R u_k  +  1/2 x_N'Q_N x_N
    s.t. x_{k+1} = A x_k + B u_k,   k = 0..N-1,   x_0 given,

plus box limits |u_k|_inf <= u_box (k = 0..N-1) and optionally |x_k|_inf <= x_box (k = 1..N).

Condensing (Sec. IV) eliminates the states. The controls are reparametrised around an
infinite-horizon LQR feedback, u_k = -K x_k + du_k, so the closed-loop matrix Abar = A - B K
drives the state recursion. Stacking y = [u_0; x_1; u_1; ...; u_{N-1}; x_N] gives
y = S du + M x_0, and the QP in du is

    P = S'HS,   q = S'HM x_0,   constraint rows G S with bounds shifted by -G M x_0,

where H = blkdiag(R, Q, R, Q, ..., R, Q_N) and G selects the limited rows of y. The QP data
that depend on x_0 are affine in it: q = F x_0, l = lo - E x_0, u = hi - E x_0.

Letters follow OSQP (P, q, A, l, u) for the QP. ``A_dyn`` is the dynamics matrix, which the
paper also calls A.

Readings of the paper used here (the paper is silent or garbled on them):
  * the decision vector is du_0..du_{N-1} and the dynamics hold for k = 0..N-1;
  * the terminal weight is Q_N = Q and the LQR gain comes from the infinite-horizon discrete
    algebraic Riccati equation with the same Q and R;
  * constraint rows are ordered all u-rows (stage-major), then all x-rows (stage-major).

Every random draw is from numpy's PCG64 generator, seeded, in a fixed documented order.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla


@dataclass
class MPCProblem:
    """A condensed MPC QP family: fixed P and A, with q, l, u affine in x_0."""

    nx: int
    nu: int
    N: int
    A_dyn: np.ndarray
    B: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    QN: np.ndarray
    K: np.ndarray  # feedback gain used for the reparametrisation (zeros = plain condensing)
    P: np.ndarray  # n x n
    F: np.ndarray  # n x nx, q = F x0
    A: np.ndarray  # m x n constraint matrix
    E: np.ndarray  # m x nx, bounds shift
    lo: np.ndarray  # m
    hi: np.ndarray  # m
    S: np.ndarray = field(repr=False, default=None)  # (N*(nu+nx)) x n, y = S du + M x0
    M: np.ndarray = field(repr=False, default=None)  # (N*(nu+nx)) x nx
    name: str = ""

    @property
    def n(self) -> int:
        return self.P.shape[0]

    @property
    def m(self) -> int:
        return self.A.shape[0]

    def instance(self, x0: np.ndarray):
        """QP vectors (q, l, u) for one initial state, or a batch of them (rows of x0)."""
        x0 = np.asarray(x0, dtype=np.float64)
        q = x0 @ self.F.T
        shift = x0 @ self.E.T
        return q, self.lo - shift, self.hi - shift

    def trajectory(self, du: np.ndarray, x0: np.ndarray):
        """Map a condensed solution back to (u_0..u_{N-1}, x_1..x_N) of the direct form."""
        y = self.S @ du + self.M @ x0
        y = y.reshape(self.N, self.nu + self.nx)
        return y[:, : self.nu], y[:, self.nu :]


def random_dynamics(nx: int, nu: int, radius: float, b_density: float, rng: np.random.Generator):
    """Gaussian A rescaled to the given spectral radius; Gaussian B, optionally masked sparse."""
    A0 = rng.standard_normal((nx, nx))
    A = A0 * (radius / np.max(np.abs(np.linalg.eigvals(A0))))
    B = rng.standard_normal((nx, nu))
    if b_density < 1.0:
        mask = rng.random((nx, nu)) < b_density
        B = B * mask
    return A, B


def lqr_gain(A: np.ndarray, B: np.ndarray, Q: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Infinite-horizon discrete LQR gain K (u = -K x) from the algebraic Riccati equation."""
    X = sla.solve_discrete_are(A, B, Q, R)
    return np.linalg.solve(R + B.T @ X @ B, B.T @ X @ A)


def condense(A, B, Q, R, QN, N, K, u_box=1.0, x_box=None, keep_maps=True):
    """Build (P, F, Acon, E, lo, hi, S, M) of the condensed QP for the reparametrisation K."""
    nx, nu = B.shape
    n = N * nu
    Abar = A - B @ K
    # state maps x_k = Sx[k] du + Mx[k] x0, k = 0..N
    Sx = np.zeros((N + 1, nx, n))
    Mx = np.zeros((N + 1, nx, nx))
    Mx[0] = np.eye(nx)
    for k in range(N):
        Sx[k + 1] = Abar @ Sx[k]
        Sx[k + 1][:, k * nu : (k + 1) * nu] += B
        Mx[k + 1] = Abar @ Mx[k]
    # control maps u_k = Su[k] du + Mu[k] x0, k = 0..N-1
    Su = -np.einsum("ij,kjn->kin", K, Sx[:N])
    for k in range(N):
        Su[k][:, k * nu : (k + 1) * nu] += np.eye(nu)
    Mu = -np.einsum("ij,kjn->kin", K, Mx[:N])

    Su2 = Su.reshape(N * nu, n)
    Mu2 = Mu.reshape(N * nu, nx)
    Sx2 = Sx[1:].reshape(N * nx, n)
    Mx2 = Mx[1:].reshape(N * nx, nx)
    Rb = np.kron(np.eye(N), R)
    Qb = np.kron(np.eye(N), Q)
    Qb[(N - 1) * nx :, (N - 1) * nx :] = QN
    P = Su2.T @ (Rb @ Su2) + Sx2.T @ (Qb @ Sx2)
    P = 0.5 * (P + P.T)
    F = Su2.T @ (Rb @ Mu2) + Sx2.T @ (Qb @ Mx2)

    rows_A = [Su2]
    rows_E = [Mu2]
    lo = [-u_box * np.ones(N * nu)]
    hi = [u_box * np.ones(N * nu)]
    if x_box is not None:
        rows_A.append(Sx2)
        rows_E.append(Mx2)
        lo.append(-x_box * np.ones(N * nx))
        hi.append(x_box * np.ones(N * nx))
    Acon = np.vstack(rows_A)
    E = np.vstack(rows_E)
    S = M = None
    if keep_maps:
        # interleave to the direct-form order y = [u_0; x_1; u_1; x_2; ...]
        S = np.concatenate([Su, Sx[1:]], axis=1).reshape(N * (nu + nx), n)
        M = np.concatenate([Mu, Mx[1:]], axis=1).reshape(N * (nu + nx), nx)
    return P, F, Acon, E, np.concatenate(lo), np.concatenate(hi), S, M


def random_mpc(
    nx: int,
    nu: int,
    N: int,
    *,
    seed: int,
    radius: float = 1.05,
    b_density: float = 1.0,
    q_kind: str = "identity",
    r_scale: float = 0.1,
    u_box: float = 1.0,
    x_box: float | None = None,
    precondition: str = "lqr",
    keep_maps: bool = True,
    name: str = "",
) -> MPCProblem:
    """Seeded random linear MPC family condensed to a dense QP.

    Draw order from ``default_rng(seed)``: A (nx*nx normals), B (nx*nu normals), the B mask
    (nx*nu uniforms, only when b_density < 1), then the Q diagonal (nx uniforms in [1, 10], only
    when q_kind == "uniform").
    """
    rng = np.random.default_rng(seed)
    A, B = random_dynamics(nx, nu, radius, b_density, rng)
    if q_kind == "identity":
        Q = np.eye(nx)
    elif q_kind == "uniform":
        Q = np.diag(rng.uniform(1.0, 10.0, nx))
    else:
        raise ValueError(q_kind)
    R = r_scale * np.eye(nu)
    QN = Q.copy()
    if precondition == "lqr":
        K = lqr_gain(A, B, Q, R)
    elif precondition == "none":
        K = np.zeros((nu, nx))
    else:
        raise ValueError(precondition)
    P, F, Acon, E, lo, hi, S, M = condense(A, B, Q, R, QN, N, K, u_box, x_box, keep_maps)
    return MPCProblem(nx, nu, N, A, B, Q, R, QN, K, P, F, Acon, E, lo, hi, S, M, name)


# Workload recipes. Sizes: n = N*nu controls, m = N*nu control-limit rows (+ N*nx state rows).
CONFIGS = {
    # single instance, FP64: n = m = 20
    "c0": dict(nx=6, nu=2, N=10, seed=0, radius=1.05, q_kind="identity", r_scale=0.1),
    # single instance, FP32: n = m = 1600, adaptive penalty over 8 values
    "c1": dict(nx=120, nu=40, N=40, seed=1, radius=1.05, q_kind="identity", r_scale=0.1),
    # humanoid-balancing-shaped: n = 600, m = 600 + 1200
    "c2": dict(nx=60, nu=30, N=20, seed=2, radius=1.02, b_density=0.3, q_kind="uniform",
               r_scale=0.01, x_box=2.0),
    # serving families, n = 200 / 800 / 1600 / 3200 (nx = 3 nu, N = 40)
    "f200": dict(nx=15, nu=5, N=40, seed=40, radius=1.05, q_kind="identity", r_scale=0.1),
    "f800": dict(nx=60, nu=20, N=40, seed=41, radius=1.05, q_kind="identity", r_scale=0.1),
    "f1600": dict(nx=120, nu=40, N=40, seed=42, radius=1.05, q_kind="identity", r_scale=0.1),
    "f3200": dict(nx=240, nu=80, N=40, seed=43, radius=1.05, q_kind="identity", r_scale=0.1),
}


def make_config(name: str, **overrides) -> MPCProblem:
    kw = dict(CONFIGS[name])
    kw.update(overrides)
    return random_mpc(name=name, **kw)


def x0_batch(nx: int, count: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """``count`` initial states x0 ~ scale * U[-1, 1]^nx from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return scale * rng.uniform(-1.0, 1.0, (count, nx))
