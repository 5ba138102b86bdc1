"""The C ABI from plain C (`paper_2311_18056_amd/capi_example.c`, built by build()): a C99
program that includes only relu_qp.h and the HIP runtime header, reads a QP from files, runs the
offline stage and one solve, and writes the results back. CPU: the program loads and rejects bad
input before any device call. GPU: its results match the oracle with the schedule replayed."""

import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import admm
from workloads import random_qp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2311_18056_amd", "relu_qp_example")


def _exe():
    if not os.path.exists(EXE):
        pytest.fail("the C example is missing: run __graft_entry__.build() first")
    return EXE


def test_c_program_rejects_bad_input(tmp_path):
    r = subprocess.run([_exe(), str(tmp_path / "missing"), "10", "0"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "dims.txt" in r.stderr
    r = subprocess.run([_exe()], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-4)])
def test_c_program_matches_the_oracle(tmp_path, prec, tol):
    P, q, A, l, u = random_qp(60, 10, 30, seed=3)
    n, m = P.shape[0], A.shape[0]
    (tmp_path / "dims.txt").write_text(f"{n} {m}\n")
    for name, v in (("P", P), ("q", q), ("A", A), ("l", l), ("u", u)):
        np.ascontiguousarray(v, dtype="<f8").tofile(tmp_path / f"{name}.bin")
    print(f"\nC example: n={n} m={m} precision={'fp64' if prec == 0 else 'fp32'}", flush=True)
    r = subprocess.run([_exe(), str(tmp_path), "150", str(prec)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    x = np.fromfile(tmp_path / "x.bin", dtype="<f8")
    z = np.fromfile(tmp_path / "z.bin", dtype="<f8")
    y = np.fromfile(tmp_path / "y.bin", dtype="<f8")
    lines = (tmp_path / "info.txt").read_text().split("\n")
    it, st = (int(t) for t in lines[0].split())
    hist = [int(t) for t in lines[1].split()]
    assert it == 150 and st == 2 and len(hist) == 6
    s = admm.Settings()
    s.n_rho, s.eps_abs, s.eps_rel, s.max_iter = 8, 0.0, 0.0, 150
    ref = oracle.solve(P, q, A, l, u, s, rho_replay=hist)
    for name, a, b in (("x", x, ref.x), ("z", z, ref.z), ("y", y, ref.y)):
        assert np.max(np.abs(a - b)) <= tol * max(np.max(np.abs(b)), 1.0), name
