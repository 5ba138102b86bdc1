"""Builds the HIP library ``librelu_qp.so`` in-tree with hipcc for gfx950.

Usage: ``python -m paper_2311_18056_amd.build`` (or ``build()`` from Python). Every call
recompiles; objects go to ``paper_2311_18056_amd/_build/``.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "librelu_qp.so")
SOURCES = ["setup_kernels.hip", "layer_kernel.hip", "batch_kernel.hip", "paper_layer.hip", "small_kernel.hip",
           "relu_qp_api.hip"]
ARCH = os.environ.get("RELU_QP_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []

    def compile_one(src):
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [hipcc, *HIP_FLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
        if verbose and msgs:
            print("\n".join(msgs))
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    build_example()
    return OUT


EXAMPLE = os.path.join(HERE, "relu_qp_example")


def build_example() -> str:
    """The plain-C user of the ABI (capi_example.c), linked against the in-tree library and the
    HIP runtime; it finds the library next to itself."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler for the C example")
    tmp = EXAMPLE + ".tmp"
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE, "-I",
           os.path.join(rocm, "include"), os.path.join(HERE, "capi_example.c"), "-L", HERE, "-lrelu_qp", "-L",
           os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(rocm, "lib"),
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C example build failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
