"""Build liblsh.so (the C-ABI library) in-tree for gfx950.

Sources are compiled with hipcc; the shared object is linked against the HIP
runtime that ships with torch, so that a process using torch for device memory
and streams holds exactly one HIP runtime (two runtimes in one process do not
share devices, streams or allocations).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblsh.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["lsh_host.cpp", "lsh_solver.hip", "lsh_twopass.hip", "lsh_unet.hip"]
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("torch is needed for its HIP runtime")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {d}")
    return d


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:  # the sources compile side by side
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *CFLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, pr in procs:
        if pr.wait() != 0:
            raise subprocess.CalledProcessError(pr.returncode, cmd)
    tl = torch_lib_dir()
    link = ["g++", "-shared", "-o", OUT + ".tmp", *objs, f"-L{tl}", "-l:libamdhip64.so",
            f"-Wl,-rpath,{tl}", "-Wl,--no-undefined"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
