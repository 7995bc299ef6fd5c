"""Writes the exact sums of the kernel-sized programs (p = 32, 64 node factors, 200 monomials)
to ``kernel_sized_p32_seed<k>.txt`` beside this file.

It calls only the oracle's term-by-term evaluator (``oracle/o2_eval.c``, binary order, full
Z[w] products, int128 with overflow traps) on the text of ``workloads.kernel_sized_program``:
the value of Eq. 2 of the paper summed over all 2^32 assignments.  About 20 minutes per seed
on 8 host threads.

    python tests/golden/make_kernel_sized.py [seed ...]      (default: 0 1)
"""

import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import o2  # noqa: E402


def golden_path(seed: int) -> str:
    return os.path.join(HERE, f"kernel_sized_p32_seed{seed}.txt")


def main(seeds):
    for seed in seeds:
        text = wl.kernel_sized_program(seed).to_text()
        t0 = time.time()
        res = o2.evaluate(text)
        dt = time.time() - t0
        z, e = res["canonical"]
        raw = res["raw"]
        with open(golden_path(seed), "w") as f:
            f.write("# exact sum of workloads.kernel_sized_program(%d) (p = 32): the oracle's\n" % seed)
            f.write("# term-by-term evaluation over all 2^32 assignments, written by make_kernel_sized.py\n")
            f.write("# ir_sha256 %s\n" % hashlib.sha256(text.encode()).hexdigest())
            f.write("# oracle wall time %.0f s on %d threads\n" % (dt, os.cpu_count() or 1))
            f.write("raw %d %d %d %d\n" % raw)
            f.write("canonical %d %d %d %d %d\n" % (z[0], z[1], z[2], z[3], e))
        print(f"seed {seed}: canonical {z} e={e} ({dt:.0f} s)", flush=True)


if __name__ == "__main__":
    main([int(s) for s in sys.argv[1:]] or [0, 1])
