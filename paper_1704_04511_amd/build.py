"""Build libslrx.so in-tree for gfx950.

Compiles every HIP source of ``csrc/`` with hipcc (offload arch gfx950) and
links the shared library against the HIP runtime, rocSOLVER and rocBLAS that
ship with the installed PyTorch, so that a process using PyTorch's device
memory and streams shares one HIP runtime with the library.

Usage: ``python -m paper_1704_04511_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libslrx.so")
SOURCES = ["k_op.hip", "k_coil.hip", "k_fit.hip", "k_gram.hip", "k_tri.hip", "k_backtr.hip", "k_dc.hip", "steps.hip", "engine.hip", "api.hip", "server.hip", "noalloc.hip", "tune.hip", "k_voxel.hip", "k_direct.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def rocm_path() -> str:
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("PyTorch is required (its HIP runtime is linked)")
    return os.path.join(list(spec.submodule_search_locations)[0], "lib")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {cmd[0]} ... {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(rocm_path(), "bin", "hipcc")
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    jobs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        jobs.append([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    tlib = torch_lib_dir()
    tmp = LIB + ".tmp"
    link = ["g++", "-shared", "-o", tmp, *objs,
            "-L", tlib, "-l:libamdhip64.so", "-l:librocsolver.so", "-l:librocblas.so",
            "-L", os.path.join(rocm_path(), "lib"), "-l:librocprofiler-sdk-roctx.so",
            f"-Wl,-rpath,{tlib}", f"-Wl,-rpath,{os.path.join(rocm_path(), 'lib')}", "-Wl,--no-undefined", "-lpthread"]
    _run(link)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
