"""Closed-loop MPC with a fixed ADMM budget per step, in FP64. TEST INFRASTRUCTURE ONLY.

The paper runs its solver inside a receding-horizon loop (Sec. V-B): at every MPC step the QP
is updated with the measured state, a fixed number of iterations is run from the previous
step's primal and dual (one per step for the random linear systems, two for the humanoid,
fifteen for the quadruped), the first control is applied to the plant, and the loop moves on.

Step k, from the state x_k:
  1. q, l, u of the condensed QP from x_k (Sec. IV; ``mpc_update.qp_vectors``);
  2. ``budget`` iterations of the ADMM (``admm.solve`` with max_iter = budget), the first step
     cold, every later one warm from the previous step's x, y and penalty index, z = A x;
  3. the applied control u_k: the first stage's constraint rows, u_k = z[0:nu] + (E x_k)[0:nu];
  4. x_{k+1} = A_d x_k + B_d u_k.

Readings (the paper gives the loop, not these details):
  * the condensed constraint rows are u = A du + E x0 with the first nu rows holding the first
    stage's control; z is their copy after the clamp, so the applied control always lies in
    the control limits, after any number of iterations;
  * a step whose budget is not a multiple of the check interval ends without a residual check
    (``final_check=False``); checks that fall inside a step run as in any solve, and the
    penalty index then chosen carries over to the next step.
"""

from __future__ import annotations

import numpy as np

from . import admm
from .mpc_update import qp_vectors


def closed_loop(P, A, F, E, lo, hi, Ad, Bd, nu: int, x0, steps: int, s: admm.Settings, cache=None):
    """Returns (xs (steps+1, nx), us (steps, nu), results of every step)."""
    if cache is None:
        cache = {}
    x = np.array(x0, np.float64)
    xs, us, results = [x.copy()], [], []
    warm = None
    for _ in range(steps):
        q, l, u = qp_vectors(F, E, lo, hi, x)
        r = admm.solve(P, q, A, l, u, s, warm=warm, cache=cache, final_check=False)
        ex = np.asarray(E, np.float64)[:nu] @ x
        uk = r.z[:nu] + ex
        x = np.asarray(Ad, np.float64) @ x + np.asarray(Bd, np.float64) @ uk
        xs.append(x.copy())
        us.append(uk)
        results.append(r)
        warm = (r.x, r.y, r.rho_index)
    return np.array(xs), np.array(us), results
