"""Builds libhtsvd.so (HIP for gfx950) in-tree with hipcc: one object per source, compiled in
parallel into a private build folder, then linked."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhtsvd.so")
SOURCES = ["api.hip", "bm.hip", "filter.hip", "filter_mfma.hip", "util.hip", "estimator.hip", "cnn.hip",
           "basis_learn.hip", "ra.hip", "bands.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay off: hipcc -O3 would otherwise form v_pk_* from scalar code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False, jobs: int = 0) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    missing = [s for s in srcs if not os.path.exists(s)]
    if missing:
        raise FileNotFoundError("missing sources: %s" % missing)
    obj_dir = os.path.join(HERE, "_build", "obj%d" % os.getpid())
    os.makedirs(obj_dir, exist_ok=True)
    objs = [os.path.join(obj_dir, os.path.basename(s)[:-4] + ".o") for s in srcs]
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 8))
    try:
        with cf.ThreadPoolExecutor(jobs) as ex:
            futs = [ex.submit(_run, [HIPCC] + FLAGS + ["-c", "-o", o, s], verbose) for s, o in zip(srcs, objs)]
            for f in futs:
                f.result()
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(obj_dir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
