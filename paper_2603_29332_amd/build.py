"""Build libms.so (HIP, gfx950) in-tree with hipcc: every source compiled to
an object in parallel, then linked."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libms.so")
SOURCES = ["ms_model.cpp", "ms_step.hip", "ms_step_v2.hip", "ms_step_v4.hip", "ms_step_v6.hip",
           "ms_step_v8.hip", "ms_step_split.hip", "ms_batch.hip", "ms_gemm.hip", "ms_mlp.hip",
           "ms_control.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # no packed-FP32 instructions in generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln)
    return r.returncode, err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source into paper_2603_29332_amd/libms.so."""
    jobs = jobs or min(len(SOURCES), max(1, len(os.sched_getaffinity(0))))
    with tempfile.TemporaryDirectory(prefix="ms_build_") as tmpd:
        objs = [os.path.join(tmpd, s + ".o") for s in SOURCES]
        cmds = [[HIPCC] + FLAGS + ["-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        for s, (rc, err) in zip(SOURCES, results):
            if rc != 0:
                sys.stderr.write(f"{s}:\n{err}\n")
                raise RuntimeError(f"hipcc failed on {s}")
            if verbose and err.strip():
                sys.stderr.write(err + "\n")
        tmp = LIB + ".tmp"
        rc, err = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
        if rc != 0:
            sys.stderr.write(err + "\n")
            raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
