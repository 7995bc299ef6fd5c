"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws random numbers and writes text: random Clifford+T circuits
(the paper's benchmark family, Section 4) and random term programs in the ``zxir 1``
text format.  It holds none of the arithmetic of the method: nothing here evaluates a
factor, a phase or a sum.  Both the oracle (``oracle/``) and the product
(``paper_2403_06777_amd``) read what these generators write; neither is imported here.
"""

from .rng import SplitMix64
from .circuits import (
    random_clifford_t,
    circuit_text,
    tiny_circuit,
    circuit_scale,
    batch_queries,
    serving_pool,
    sampling_circuit,
    sampling_uniforms,
)
from .programs import (
    ProgramSpec,
    kernel_sized_program,
    random_program,
    block_separable_program,
    appendix_d_terms,
    weight4_phase_program,
    block_bound_program,
)

__all__ = [
    "SplitMix64",
    "random_clifford_t",
    "circuit_text",
    "tiny_circuit",
    "circuit_scale",
    "batch_queries",
    "serving_pool",
    "sampling_circuit",
    "sampling_uniforms",
    "ProgramSpec",
    "kernel_sized_program",
    "random_program",
    "block_separable_program",
    "appendix_d_terms",
    "weight4_phase_program",
    "block_bound_program",
]
