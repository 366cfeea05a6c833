"""Compile the HIP library (gfx950) into paper_1501_03879_amd/libemx.so.

Each .hip source is compiled to an object in parallel, then linked with
hipcc -shared.  Packed-FP32 instructions are disabled for every device
compile (target feature -packed-fp32-ops).
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.environ.get("EMX_BUILD_OUTPUT") or os.path.join(HERE, "libemx.so")
BUILD_DIR = os.environ.get("EMX_BUILD_DIR") or os.path.join(HERE, "_build")
SOURCES = ["nlem_pr0.hip", "nlem_pr1.hip", "nlem_pr2.hip", "nlem_pr3.hip", "batch_admm.hip",
           "batch_irls.hip", "batch_adapt.hip", "batch_admm_ball.hip", "batch_irls_ball.hip",
           "batch_wpen.hip", "batch_wpen_ball.hip", "batch_wide.hip", "batch_fast.hip",
           "batch_host.hip", "nlem_order.hip",
           "emx_host.hip"]
ARCH = os.environ.get("EMX_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def compile_flags():
    extra = os.environ.get("EMX_EXTRA_FLAGS", "").split()
    return extra + [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Wno-unused-result", "-Wno-unused-variable",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(HERE, "..", "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + compile_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    if errs.strip():
        sys.stderr.write(errs + "\n")
    return obj


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    build_client()
    return LIB


CLIENT_SRC = os.path.join(HERE, "examples", "nlem_client.c")
CLIENT = os.path.join(HERE, "examples", "nlem_client")


def build_client() -> str:
    """The C example client (examples/nlem_client.c): plain C against
    include/emx.h and the HIP runtime, linked to libemx.so in this directory."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(HERE, "..", "include"),
           CLIENT_SRC, "-o", CLIENT, "-L", os.path.dirname(LIB), "-l:" + os.path.basename(LIB),
           "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed for the C client:\n" + r.stdout + r.stderr)
    return CLIENT


if __name__ == "__main__":
    print(build())
