"""Compile libknn.so (HIP, gfx950) in-tree.

    python -m paper_1607_08220_amd.build [--incremental]

Every source is compiled with ``-ffp-contract=off`` (no fused multiply-add:
the FP32 distance is defined with a separate multiply and add) and without
flushing denormals, plus ``-packed-fp32-ops`` disabled (no v_pk_* FP32 ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libknn.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = ["knn_api.hip", "knn_build.hip", "knn_query.hip", "knn_trav_lane1.hip",
           "knn_trav_lane2.hip", "knn_trav_stack1.hip", "knn_trav_stack2.hip", "knn_trav_team.hip",
           "knn_serve.hip",
           "knn_classify.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("KNN_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}",
]


def _newest_dependency(src: str) -> float:
    deps = [os.path.join(CSRC, src), os.path.join(CSRC, "knn_internal.h"),
            os.path.join(INCLUDE, "knn.h"), os.path.abspath(__file__)]
    if '#include "knn_traverse.h"' in open(deps[0]).read():
        deps.append(os.path.join(CSRC, "knn_traverse.h"))
    return max(os.path.getmtime(p) for p in deps)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _newest_dependency(src):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    errs = [l for l in r.stderr.splitlines()
            if l.strip() and "packed-fp32-ops" not in l]
    if errs:
        sys.stderr.write("\n".join(errs) + "\n")
    return obj


def compile_library(out: str = LIB, incremental: bool = False) -> str:
    """Compile every source (``incremental``: only those whose object is
    older than the source or a shared header) and link the library."""
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, incremental), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(compile_library(incremental="--incremental" in sys.argv))
