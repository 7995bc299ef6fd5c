"""Python driver of the term-by-term evaluator ``o2_eval.c``: TEST INFRASTRUCTURE ONLY.

Builds the C program with gcc (plain C, no GPU), feeds it a ``zxir 1`` program text and
parses its exact output.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg use this module.
"""

import os
import subprocess
from typing import Optional, Sequence, Tuple

from . import zomega as zw

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "o2_eval.c")
EXE = os.path.join(HERE, "o2_eval")


def build(force: bool = False) -> str:
    if force or not os.path.exists(EXE) or os.path.getmtime(EXE) < os.path.getmtime(SRC):
        tmp = EXE + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-Wall", "-pthread", "-o", tmp, SRC],
                       check=True)
        os.replace(tmp, EXE)
    return EXE


class OracleOverflow(RuntimeError):
    pass


def evaluate(ir_text: str, threads: Optional[int] = None, first: Optional[int] = None,
             count: Optional[int] = None, perm: Optional[Sequence[int]] = None,
             terms: bool = False, timeout: Optional[float] = None,
             points: Optional[Tuple[int, Sequence[int]]] = None) -> dict:
    """Returns {'raw': sum without scalar, 'value': (c * sum, e), 'canonical': (z, e),
    'terms': {index: z}}.  points = (x0, cols): index t is the assignment x0 ^ (xor of cols[j]
    over the set bits j of t) instead of a relabelling of 0 .. 2^p - 1."""
    exe = build()
    args = [exe, "--threads", str(threads or os.cpu_count() or 1)]
    if first is not None or count is not None:
        args += ["--first", str(first or 0), "--count", str(count)]
    if perm is not None:
        args += ["--perm", ",".join(str(v) for v in perm)]
    if points is not None:
        x0, cols = points
        args += ["--points", ",".join("%x" % v for v in [x0] + list(cols))]
    if terms:
        args.append("--terms")
    proc = subprocess.run(args, input=ir_text, capture_output=True, text=True, timeout=timeout)
    if proc.returncode == 3:
        raise OracleOverflow(proc.stderr.strip())
    if proc.returncode != 0:
        raise RuntimeError(f"o2_eval failed ({proc.returncode}): {proc.stderr.strip()}")
    out = {"terms": {}}
    for line in proc.stdout.splitlines():
        tok = line.split()
        if tok[0] == "raw":
            out["raw"] = tuple(int(v) for v in tok[1:5])
        elif tok[0] == "value":
            out["value"] = (tuple(int(v) for v in tok[1:5]), int(tok[5]))
        elif tok[0] == "term":
            out["terms"][int(tok[1])] = tuple(int(v) for v in tok[2:6])
    out["canonical"] = zw.canonical(*out["value"])
    return out
