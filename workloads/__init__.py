"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds problem data only. It holds none of the ADMM arithmetic: no KKT inverse,
no layer step, no residual, no penalty rule. Both the CPU oracle (``oracle/``) and the HIP
path (``paper_2311_18056_amd``) take its output as input; neither side's code lives here.
"""

from .mpc import (  # noqa: F401
    MPCProblem,
    CONFIGS,
    make_config,
    random_mpc,
    x0_batch,
)
from .dense import random_qp, random_box_qp  # noqa: F401
