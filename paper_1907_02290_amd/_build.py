"""Build ``libnbody_hip.so`` (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled with packed-FP32 instructions disabled.
The tree, walk, integration and refresh units are also compiled without
floating-point contraction (the rounding intrinsics are plain operations
that the compiler could otherwise fuse), because keys, cell centres, boxes,
the opening test and the position update must be bit-identical to an FP64
reference.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnbody_hip.so")
ARCH = "gfx950"

SOURCES = ["nb_scan.hip", "nb_tree.hip", "nb_walk.hip", "nb_force.hip",
           "nb_step.hip", "nb_learn.hip", "nb_api.hip"]
EXACT = {"nb_tree.hip", "nb_walk.hip", "nb_step.hip", "nb_learn.hip"}

COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = ["hipcc", *COMMON]
    if src in EXACT:
        cmd.append("-ffp-contract=off")
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout,
                                                             r.stderr))
    return obj


def build(jobs: int = 6, verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs,
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
