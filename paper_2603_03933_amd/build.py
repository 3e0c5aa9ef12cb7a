"""Build liblbtr.so, the HIP library behind include/lb.h, for gfx950.

Every FFT length is compiled in its own translation unit (csrc/inst.hip with
-DLB_N=<length>) in parallel, then linked with the main unit csrc/lb_lib.hip.
The library binds to the HIP runtime that PyTorch ships (the process's torch
import loads it first; the RUNPATH lets a torch-free process find the same
runtime) so that one runtime serves both.

Usage: python -m paper_2603_03933_amd.build  (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import importlib.util
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbtr.so")
LENGTHS = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512)
ARCH = os.environ.get("LB_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _torch_lib() -> str:
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("torch is required: its HIP runtime is the one the library binds to")
    return os.path.join(os.path.dirname(spec.origin), "lib")


def _flags():
    return [
        "-std=c++17",
        "-O3",
        f"--offload-arch={ARCH}",
        "-fPIC",
        # no packed FP32 instructions in generated code
        "-Xclang",
        "-target-feature",
        "-Xclang",
        "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
    ]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP translation unit and link liblbtr.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    fl = _flags()
    jobs = jobs or min(16, os.cpu_count() or 4)
    cmds = []
    for n in LENGTHS:
        cmds.append([hipcc, *fl, f"-DLB_N={n}", "-c", os.path.join(CSRC, "inst.hip"), "-o", os.path.join(BUILD, f"inst_{n}.o")])
    cmds.append([hipcc, *fl, "-c", os.path.join(CSRC, "lb_lib.hip"), "-o", os.path.join(BUILD, "lb_lib.o")])
    with cf.ThreadPoolExecutor(jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tl = _torch_lib()
    objs = [os.path.join(BUILD, f"inst_{n}.o") for n in LENGTHS] + [os.path.join(BUILD, "lb_lib.o")]
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-o", tmp, *objs, f"-L{tl}", "-l:libamdhip64.so", f"-Wl,-rpath,{tl}:/opt/rocm/lib", "-Wl,--no-undefined"])
    os.replace(tmp, LIB)
    _build_c_client(tl)
    return LIB


def _build_c_client(torch_lib: str) -> None:
    """The plain-C test client of the ABI (tests/c/lb_client.c), if present,
    linked against liblbtr.so and the same HIP runtime."""
    root = os.path.dirname(HERE)
    src = os.path.join(root, "tests", "c", "lb_client.c")
    if not os.path.exists(src):
        return
    exe = os.path.join(root, "tests", "c", "lb_client")
    _run(["gcc", "-O2", "-std=c11", f"-I{os.path.join(root, 'include')}", src, "-o", exe, f"-L{HERE}", "-llbtr",
          f"-L{torch_lib}", "-l:libamdhip64.so", f"-Wl,-rpath,{HERE}:{torch_lib}:/opt/rocm/lib", "-lm"])


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
