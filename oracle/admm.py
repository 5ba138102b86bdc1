"""FP64 oracle of the ReLU-QP ADMM iteration. TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Problem (paper Sec. II-A, eq. qp_def):  min 1/2 x'Px + q'x  s.t.  l <= A x <= u.

Letters follow OSQP. The paper writes (H, g, G, c, d) for (P, q, A, l, u); its primal y is x
here, its constraint copy z is z, and its constraint multiplier lambda is y here.

Three forms of one iteration are kept, so that each pins the others:

* ``step_T`` -- ADMM as in OSQP's Algorithm 1 (the ADMM the paper cites in Sec. II-B), with the
  full quasi-definite KKT system solved by LU, and OSQP's over-relaxation alpha.
* ``step_R`` -- the same iteration in "layer" form, with the explicit inverse
  D = (P + sigma I + A' diag(rho) A)^-1 of Sec. III-A (the matrix called D under eq.
  gpu_update): a dense matvec followed by a clamp. This is the form the GPU path computes.
* ``step_L`` -- the paper's literal weight-tied layer v+ = clamp(W v + b) of eq. gpu_update,
  with W and b built block by block as printed (alpha = 1, fixed rho only).
* ``step_paper5`` -- the five-variable iteration of eqs. Xbar_update..lambda_update_gen (alpha = 1),
  kept to pin the paper's remark that mu vanishes after one iteration.

Readings of the paper (it is silent or ambiguous on these):
  * over-relaxation alpha in (0, 2) is OSQP's; alpha = 1 reproduces the paper's iteration;
  * the state is the textbook (x, z, y); the paper's layer carries a dual lagged by one step,
    which agrees with the textbook only at alpha = 1 and fixed rho (tested);
  * the stopping test uses OSQP's mixed tolerances eps_abs + eps_rel * max(norms), inf-norms,
    and "<=" (eqs. primal and dual);
  * the penalty grid is log-spaced rho_min..rho_max (Sec. III-C, penalty heuristics); the
    starting value rho0 is replaced by the nearest grid value in log distance (ties to the
    smaller value); the rule of eq. rho_update is evaluated from the active grid value and
    rounded to the nearest grid value; it is skipped when either residual is zero;
  * the check runs every ``check_interval`` iterations and at ``max_iter``; residuals first,
    then the penalty update if not converged;
  * rows with l_i == u_i get a penalty rho_eq_scale times larger (Sec. II-B);
  * eps_abs == eps_rel == 0 turns the convergence test off (fixed-iteration mode);
  * a non-finite norm ends the solve with status NONFINITE.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

RUNNING, SOLVED, MAX_ITER, NONFINITE, ABORTED = 0, 1, 2, 3, 4


@dataclass
class Settings:
    sigma: float = 1e-6
    alpha: float = 1.6
    rho0: float = 0.1
    n_rho: int = 1
    rho_min: float = 1e-3
    rho_max: float = 1e3
    rho_eq_scale: float = 1e3
    eps_abs: float = 1e-3
    eps_rel: float = 1e-3
    max_iter: int = 4000
    check_interval: int = 25


@dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    iterations: int
    status: int
    rho_index: int
    rho_hist: list = field(default_factory=list)  # grid index in force after each check
    prim_res: list = field(default_factory=list)
    dual_res: list = field(default_factory=list)
    history: list | None = None  # (x, z, y) after every iteration when recorded


# ----------------------------------------------------------------------------------------------
# penalty grid (Sec. III-C, "Penalty Scaling Heuristics"; eq. rho_update)


def rho_grid(s: Settings) -> np.ndarray:
    """Grid of penalty values: {rho0} for a fixed penalty, else log-spaced rho_min..rho_max."""
    if s.n_rho == 1:
        return np.array([float(s.rho0)])
    lo, hi = np.log10(s.rho_min), np.log10(s.rho_max)
    return 10.0 ** (lo + np.arange(s.n_rho) * (hi - lo) / (s.n_rho - 1))


def nearest_rho_index(grid: np.ndarray, rho: float) -> int:
    """Index of the grid value closest to rho in log distance; ties go to the smaller value."""
    d = np.abs(np.log(grid) - np.log(rho))
    return int(np.argmin(d))  # argmin returns the first (smallest) index on ties


def rho_start_index(s: Settings) -> int:
    return 0 if s.n_rho == 1 else nearest_rho_index(rho_grid(s), s.rho0)


def rho_vector(rho_bar: float, eq: np.ndarray, s: Settings) -> np.ndarray:
    """Diagonal penalty: rho_bar on inequality rows, rho_eq_scale * rho_bar on equality rows."""
    return np.where(eq, s.rho_eq_scale * rho_bar, rho_bar).astype(np.float64)


def rho_hat(rho_bar: float, n: dict) -> float:
    """Nominal penalty of eq. rho_update from the check's norms (dict from residual_norms)."""
    num = n["r_p"] * max(n["Px"], n["Aty"], n["q"], 1e-4)
    den = n["r_d"] * max(n["Ax"], n["z"], 1e-4)
    return rho_bar * np.sqrt(num / den)


# ----------------------------------------------------------------------------------------------
# the projection (eq. clamp) and its two-ReLU form


def clamp(t: np.ndarray, l: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Projection onto the box [l, u]; NaN propagates."""
    return np.minimum(np.maximum(t, l), u)


def relu(v: np.ndarray) -> np.ndarray:
    return np.where(v > 0, v, 0.0)


def clamp_two_relu(t, l, u):
    """t - ReLU(t - u) + ReLU(l - t): the clamp written with two ReLUs (finite t, l, u)."""
    return t - relu(t - u) + relu(l - t)


# ----------------------------------------------------------------------------------------------
# offline setup: the KKT inverse (Sec. III-A, D below eq. gpu_update; Algorithm 1, offline)


def kkt_matrix(P, A, sigma, rho_vec):
    n = P.shape[0]
    return P + sigma * np.eye(n) + A.T @ (rho_vec[:, None] * A)


def kkt_inverse(P, A, sigma, rho_vec):
    """D = (P + sigma I + A' diag(rho) A)^-1 through a Cholesky factorisation.

    Raises numpy.linalg.LinAlgError when the matrix is not positive definite.
    """
    K = kkt_matrix(P, A, sigma, rho_vec)
    c = sla.cho_factor(K, lower=True)
    D = sla.cho_solve(c, np.eye(K.shape[0]))
    return 0.5 * (D + D.T)


# ----------------------------------------------------------------------------------------------
# one iteration, three ways


def step_R(x, z, y, D, rho_vec, q, A, l, u, sigma, alpha):
    """Layer form with the explicit inverse D (the form the GPU path computes).

    xt = D (sigma x - q + A'(rho z - y))          (eq. Xbar_update with mu = 0)
    x+ = alpha xt + (1 - alpha) x                   (relaxation)
    t  = alpha A xt + (1 - alpha) z + y / rho
    z+ = clamp(t, l, u)                             (eq. z_update)
    y+ = rho (t - z+)                               (eq. lambda_update_gen, relaxed)
    """
    xt = D @ (sigma * x - q + A.T @ (rho_vec * z - y))
    x_new = alpha * xt + (1.0 - alpha) * x
    t = alpha * (A @ xt) + (1.0 - alpha) * z + y / rho_vec
    z_new = clamp(t, l, u)
    y_new = rho_vec * (t - z_new)
    return x_new, z_new, y_new


def step_T(x, z, y, kkt_lu, rho_vec, q, A, l, u, sigma, alpha):
    """OSQP's ADMM step (its Algorithm 1): full KKT solve, then relaxed z and y updates.

    [P + sigma I, A'; A, -diag(1/rho)] [xt; nu] = [sigma x - q; z - y/rho]
    zt = z + (nu - y)/rho;  x+ = alpha xt + (1-alpha) x
    z+ = clamp(alpha zt + (1-alpha) z + y/rho);  y+ = y + rho (alpha zt + (1-alpha) z - z+)
    """
    n = x.shape[0]
    rhs = np.concatenate([sigma * x - q, z - y / rho_vec])
    sol = sla.lu_solve(kkt_lu, rhs)
    xt, nu = sol[:n], sol[n:]
    zt = z + (nu - y) / rho_vec
    x_new = alpha * xt + (1.0 - alpha) * x
    zr = alpha * zt + (1.0 - alpha) * z
    z_new = clamp(zr + y / rho_vec, l, u)
    y_new = y + rho_vec * (zr - z_new)
    return x_new, z_new, y_new


def full_kkt_lu(P, A, sigma, rho_vec):
    n, m = P.shape[0], A.shape[0]
    K = np.zeros((n + m, n + m))
    K[:n, :n] = P + sigma * np.eye(n)
    K[:n, n:] = A.T
    K[n:, :n] = A
    K[n:, n:] = -np.diag(1.0 / rho_vec)
    return sla.lu_factor(K)


def step_paper5(ybar, y, z, mu, lam, D, rho_vec, H, g, G, c, d, sigma):
    """The paper's five-variable ADMM step, eqs. Xbar_update, x_update, z_update,
    mu_update_gen, lambda_update_gen, in the paper's own letters (alpha = 1)."""
    ybar_n = D @ (-g + sigma * y - mu + G.T @ (rho_vec * z - lam))
    y_n = ybar_n + mu / sigma
    z_n = clamp(G @ ybar_n + lam / rho_vec, c, d)
    mu_n = mu + sigma * (ybar_n - y_n)
    lam_n = lam + rho_vec * (G @ y_n - z_n)
    return ybar_n, y_n, z_n, mu_n, lam_n


def paper_W(D, H, G, rho_vec, sigma):
    """The weight matrix W of eq. gpu_update, block by block as printed (diagonal rho)."""
    n, m = H.shape[0], G.shape[0]
    Rm = np.diag(rho_vec)
    Ri = np.diag(1.0 / rho_vec)
    I_n, I_m = np.eye(n), np.eye(m)
    GtRG = G.T @ Rm @ G
    W = np.zeros((n + 2 * m, n + 2 * m))
    W[:n, :n] = D @ (sigma * I_n - GtRG)
    W[:n, n : n + m] = 2.0 * D @ G.T @ Rm
    W[:n, n + m :] = -D @ G.T
    W[n : n + m, :n] = G @ D @ (sigma * I_n - GtRG) + G
    W[n : n + m, n : n + m] = 2.0 * G @ D @ G.T @ Rm - I_m
    W[n : n + m, n + m :] = -G @ D @ G.T + Ri
    W[n + m :, :n] = Rm @ G
    W[n + m :, n : n + m] = -Rm
    W[n + m :, n + m :] = I_m
    return W


def paper_b(D, G, g):
    """The bias b = [-D; -GD; 0] g of eq. gpu_update."""
    m = G.shape[0]
    return np.concatenate([-D @ g, -G @ (D @ g), np.zeros(m)])


def step_L(v, W, b, n, m, c, d):
    """One layer v+ = clamp(W v + b, c~, d~): only the z block is clamped (eq. gpu_update)."""
    s = W @ v + b
    s[n : n + m] = clamp(s[n : n + m], c, d)
    return s


# ----------------------------------------------------------------------------------------------
# convergence check (eqs. primal, dual) and the solve loop (Algorithm 1)


def _ninf(v) -> float:
    v = np.asarray(v)
    return float(np.max(np.abs(v))) if v.size else 0.0


def residual_norms(P, q, A, x, z, y) -> dict:
    """The inf-norms the check needs: residuals r_p, r_d and the scale terms."""
    Ax = A @ x
    Px = P @ x
    Aty = A.T @ y
    return dict(
        r_p=_ninf(Ax - z),
        r_d=_ninf(Px + q + Aty),
        Ax=_ninf(Ax),
        z=_ninf(z),
        Px=_ninf(Px),
        Aty=_ninf(Aty),
        q=_ninf(q),
    )


def _validate(P, q, A, l, u, s):
    n = P.shape[0]
    m = A.shape[0]
    if P.shape != (n, n) or A.shape != (m, n) or q.shape != (n,) or l.shape != (m,) or u.shape != (m,):
        raise ValueError("inconsistent shapes")
    if n < 1 or m < 1:
        raise ValueError("need n >= 1 and m >= 1")
    if not (np.all(np.isfinite(P)) and np.all(np.isfinite(A))):
        raise ValueError("P and A must be finite")
    if np.any(l > u):
        raise ValueError("l > u")
    if not (0.0 < s.alpha < 2.0) or s.sigma <= 0.0 or s.n_rho < 1 or s.max_iter < 1 or s.check_interval < 1:
        raise ValueError("bad settings")


def solve(P, q, A, l, u, s: Settings, *, form: str = "R", warm=None, rho_replay=None, record=False,
          cache: dict | None = None, final_check: bool = True, original=None) -> Result:
    """ReLU-QP solve (Algorithm 1, online part), in FP64.

    ``warm``: None for a cold start (x = z = y = 0), or (x, y, rho_index): the previous primal,
    dual and penalty, with z = A x (Sec. II-B, warm starting).
    ``rho_replay``: optional list of grid indices; at check number c the solver takes
    rho_replay[c] instead of evaluating the penalty rule (used to replay another solver's
    schedule).
    ``cache``: optional dict that keeps the factorisations of the offline stage between calls
    on the same P, A, settings and equality pattern (Algorithm 1 computes them once).
    ``final_check=False``: a max_iter that is not a multiple of check_interval ends the solve
    with MAX_ITER and no check (a fixed iteration budget per MPC step, Sec. V-B).
    ``original``: for a scaled problem (``scaling.scale_problem``), the tuple
    (P0, q0, A0, D, E, c) of the original data and the scaling: the check then evaluates the
    residuals and norms of the original problem at the unscaled iterates.
    """
    P = np.asarray(P, np.float64)
    q = np.asarray(q, np.float64)
    A = np.asarray(A, np.float64)
    l = np.asarray(l, np.float64)
    u = np.asarray(u, np.float64)
    _validate(P, q, A, l, u, s)
    n, m = P.shape[0], A.shape[0]
    grid = rho_grid(s)
    eq = l == u
    terminate = not (s.eps_abs == 0.0 and s.eps_rel == 0.0)

    if warm is None:
        x, y, z = np.zeros(n), np.zeros(m), np.zeros(m)
        j = rho_start_index(s)
    else:
        x = np.array(warm[0], np.float64)
        y = np.array(warm[1], np.float64)
        j = int(warm[2])
        z = A @ x

    if cache is None:
        cache = {}

    def op(jj):
        jj = (form, jj)
        if jj not in cache:
            rv = rho_vector(grid[jj[1]], eq, s)
            if form == "R":
                cache[jj] = (kkt_inverse(P, A, s.sigma, rv), rv)
            elif form == "T":
                cache[jj] = (full_kkt_lu(P, A, s.sigma, rv), rv)
            else:
                raise ValueError(form)
        return cache[jj]

    res = Result(x, y, z, 0, RUNNING, j, history=[] if record else None)
    n_check = 0
    for k in range(1, s.max_iter + 1):
        M, rv = op(j)
        if form == "R":
            x, z, y = step_R(x, z, y, M, rv, q, A, l, u, s.sigma, s.alpha)
        else:
            x, z, y = step_T(x, z, y, M, rv, q, A, l, u, s.sigma, s.alpha)
        if record:
            res.history.append((x.copy(), z.copy(), y.copy()))
        if k % s.check_interval != 0 and k != s.max_iter:
            continue
        if k % s.check_interval != 0 and not final_check:
            res.status = MAX_ITER
            res.iterations = k
            break
        if original is None:
            nm = residual_norms(P, q, A, x, z, y)
        else:
            P0, q0, A0, D, E, c = original
            nm = residual_norms(P0, q0, A0, D * x, z / E, E * y / c)
        res.prim_res.append(nm["r_p"])
        res.dual_res.append(nm["r_d"])
        status = RUNNING
        if not all(np.isfinite(v) for v in nm.values()):
            status = NONFINITE
        elif terminate:
            eps_p = s.eps_abs + s.eps_rel * max(nm["Ax"], nm["z"])
            eps_d = s.eps_abs + s.eps_rel * max(nm["Px"], nm["Aty"], nm["q"])
            if nm["r_p"] <= eps_p and nm["r_d"] <= eps_d:
                status = SOLVED
        if status == RUNNING and k == s.max_iter:
            status = MAX_ITER
        if status == RUNNING:
            if rho_replay is not None:
                j = int(rho_replay[n_check])
            elif s.n_rho > 1 and nm["r_p"] > 0.0 and nm["r_d"] > 0.0:
                j = nearest_rho_index(grid, rho_hat(grid[j], nm))
        res.rho_hist.append(j)
        n_check += 1
        if status != RUNNING:
            res.status = status
            res.iterations = k
            break
    res.x, res.y, res.z, res.rho_index = x, y, z, j
    return res
