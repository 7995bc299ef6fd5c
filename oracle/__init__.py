"""Independent CPU oracle of the parametric ZX evaluation path: TEST INFRASTRUCTURE ONLY.

* ``o2_eval.c`` / ``o2.py``: term-by-term evaluator of a term program (plain C, int128,
  binary enumeration order, full Z[w] products).
* ``statevector.py``: exact Z[w] state-vector simulator (amplitudes, marginals) and a
  complex128 variant for tolerance checks.
* ``zomega.py``: exact Z[w] arithmetic and the canonical form used to compare scalars.
* ``sampling.py``: repeated weak simulation by the chain rule on the exact distribution.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use this package.
It imports nothing from the GPU library, and the GPU library never imports it.
"""
