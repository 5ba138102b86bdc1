"""Plain, slow FP64 CPU oracle of the ReLU-QP method (arXiv 2311.18056).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import or call anything here. The library under
``paper_2311_18056_amd`` never imports it, and this package never imports that library: the two
share no code. Inputs come from the seeded generators in ``workloads/``.

Modules:
  * ``admm``       -- the ADMM iteration in three equivalent forms, residuals, penalty rule, solve
  * ``bruteforce`` -- exact QP solution by active-set enumeration (tiny problems)
  * ``lqr``        -- finite-horizon Riccati recursion (exact unconstrained MPC solution)
  * ``mpc_update`` -- the per-solve QP vectors of a condensed MPC problem from x0
  * ``closed_loop`` -- receding-horizon MPC with a fixed ADMM budget per step and a plant
  * ``scaling``    -- modified Ruiz equilibration with cost scaling, unscaled termination

Parity pins: every function is pinned by a ``-m "not gpu"`` test against something other than
itself (closed forms, brute force, the paper's own matrix W, Riccati). The iteration counts and
run times are "parity unpinned": the paper prints no iterates and no counts.
"""

from .admm import (  # noqa: F401
    ABORTED,
    MAX_ITER,
    NONFINITE,
    RUNNING,
    SOLVED,
    Result,
    Settings,
    clamp,
    kkt_inverse,
    nearest_rho_index,
    residual_norms,
    rho_grid,
    rho_hat,
    rho_start_index,
    rho_vector,
    solve,
    step_L,
    step_R,
    step_T,
    step_paper5,
    paper_W,
)
