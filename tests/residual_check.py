"""The FP64 stopping test (eqs. primal, dual) evaluated on the CPU for a solution the GPU
returned: every solution the GPU declares SOLVED must pass it exactly (1.0 x eps), whatever its
iteration precision. Helpers for the GPU tests; the residuals come from the oracle."""

from oracle import admm


def eps_ratios(P, q, A, x, z, y, eps_abs=1e-3, eps_rel=1e-3):
    """(r_p / eps_p, r_d / eps_d) of the FP64 test at (x, z, y)."""
    nm = admm.residual_norms(P, q, A, x, z, y)
    eps_p = eps_abs + eps_rel * max(nm["Ax"], nm["z"])
    eps_d = eps_abs + eps_rel * max(nm["Px"], nm["Aty"], nm["q"])
    return nm["r_p"] / eps_p, nm["r_d"] / eps_d


def assert_passes_fp64_test(P, q, A, x, z, y, eps_abs=1e-3, eps_rel=1e-3, what=""):
    """Assert that (x, z, y) passes the FP64 test at 1.0 x eps; prints and returns the worse ratio."""
    rp, rd = eps_ratios(P, q, A, x, z, y, eps_abs, eps_rel)
    worst = max(rp, rd)
    print(f"\n{what}: FP64 test ratios r_p/eps_p = {rp:.4f}, r_d/eps_d = {rd:.4f}")
    assert rp <= 1.0 and rd <= 1.0, f"{what}: fails the FP64 test (r_p/eps_p {rp:.6f}, r_d/eps_d {rd:.6f})"
    return worst
