"""Compile the HIP library libragsnn.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libragsnn.so")
SOURCES = ["engine.hip", "k_build.hip", "k_forward.hip", "k_eprop.hip", "k_update.hip", "k_deepr.hip", "k_topo.hip", "k_topo_sim.hip", "k_topo_tiles.hip", "k_serve.hip", "k_custom.hip", "noalloc.hip"]
HEADERS = ["rs_device.hpp", "rs_kernels.hpp", "rs_compact.hpp", "rs_custom.hpp", "rs_host_rng.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every multiply-add is rounded as written (or is an explicit fma): the
    # compiler may not fuse differently in different instantiations of a kernel
    "-ffp-contract=off",
    # packed FP32 instructions stay disabled in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-o", tmp] + \
        [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libragsnn.so")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    srcs = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    srcs.append(os.path.join(HERE, "..", "include", "ragsnn.h"))
    return any(os.path.getmtime(s) > t for s in srcs)


if __name__ == "__main__":
    print(build(verbose=True))
