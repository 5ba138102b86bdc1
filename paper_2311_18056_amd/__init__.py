"""MI355X (gfx950) ReLU-QP: the ADMM iteration of arXiv 2311.18056 as a persistent HIP kernel.

``Solver`` wraps the C ABI of ``include/relu_qp.h``; the shared library is built in-tree with
``python -m paper_2311_18056_amd.build``. torch is imported first so that the HIP runtime it
loads is the one the library binds to (both use the soname libamdhip64.so.7).
"""

import torch  # noqa: F401  (loads the process's HIP runtime before the library)

from ._lib import (  # noqa: F401
    RQP_ABORTED,
    RQP_BF16X3,
    RQP_FP32,
    RQP_FP64,
    RQP_IDLE,
    RQP_INTERNAL,
    RQP_MAX_ITER,
    RQP_NONFINITE,
    RQP_RUNNING,
    RQP_SOLVED,
    ReluQPError,
    lib,
)
from .solver import STATUS_NAMES, Solver, close_all, default_settings, footprint, open_handles  # noqa: F401
