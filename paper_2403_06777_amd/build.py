"""Builds libzxpar.so for gfx950 with hipcc (in-tree, next to this file)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libzxpar.so")
# the evaluation kernels are instantiated per form-vector width and monomial flag, one unit
# each, largest first so that the parallel build finishes early
SOURCES = ["eval_w16_m1.hip", "eval_w16_m0.hip", "eval_w8_m1.hip", "eval_w8_m0.hip", "eval_w4_m1.hip",
           "eval_w4_m0.hip", "eval_w2_m1.hip", "eval_w2_m0.hip", "eval_w1_m1.hip", "eval_w1_m0.hip",
           "kernels.hip", "capi.cpp", "program.cpp", "compiler.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-fvisibility=hidden",
    # no packed fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source to an object in parallel (up to `jobs` at once, default: the
    CPU count, at most 16), then links the shared library."""
    objdir = os.path.join(HERE, "_objs")
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 1)
    cmds = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmds.append([HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)])
    running, failed = [], []
    pending = list(cmds)
    while pending or running:
        while pending and len(running) < jobs:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                  text=True)))
        cmd, proc = running.pop(0)
        out, _ = proc.communicate()
        if proc.returncode != 0:
            failed.append((cmd, out))
    if failed:
        for cmd, out in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + out)
        raise RuntimeError("hipcc failed building libzxpar.so")
    tmp = OUT + ".tmp"
    objs = [c[c.index("-o") + 1] for c in cmds]
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    proc = subprocess.run(link, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("linking libzxpar.so failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
