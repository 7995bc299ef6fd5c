"""Exact MI355X evaluation of parametric ZX-calculus scalars (Sutcliffe & Kissinger, QPL 2024).

The C-ABI library ``libzxpar.so`` (hand-written HIP kernels for gfx950) does all the work;
``binding`` exposes each entry point under its C name, and ``Program`` is a small owner of a
program handle.  Nothing here computes: if the library is missing, calls raise.
"""

from . import binding
from .binding import (  # noqa: F401
    SimError,
    amplitude_query,
    marginal_query,
    outcomes_query,
    prefix_query,
    sim_batch_forget,
    sim_batch_plan_create,
    sim_batch_plan_free,
    sim_batch_plan_run,
    sim_compile,
    sim_compile_to_ir,
    sim_device_cus,
    sim_enqueue_amplitude,
    sim_eval_amplitude,
    sim_eval_amplitude_ws,
    sim_eval_batch_ws,
    sim_eval_range_ws,
    sim_enqueue_batch,
    sim_batch_prepare,
    sim_scratch_bytes,
    zomegas_from_bytes,
    sim_eval_batch,
    sim_eval_range,
    sim_eval_timed,
    sim_eval_outcomes,
    sim_eval_ranges,
    sim_eval_ranges_static,
    sim_finalize,
    sim_finalize_batch,
    sim_init,
    sim_ir_info,
    sim_ir_affine_layout,
    sim_last_error,
    sim_marginal_sum,
    sim_program_free,
    sim_program_from_ir,
    sim_program_from_ir_flags,
    sim_ir_info_flags,
    sim_program_info,
    sim_program_ir,
    sim_program_layout,
    sim_program_affine_layout,
    sim_raw_add,
    sim_sample,
    sim_serve_step,
    sim_serve_enqueue,
    zomega_from_bytes,
)


class Program:
    """Owns one compiled or parsed program on the current device."""

    def __init__(self, handle: int):
        self.handle = handle

    @classmethod
    def from_ir(cls, ir_text: str) -> "Program":
        return cls(sim_program_from_ir(ir_text))

    @classmethod
    def compile_amplitude(cls, circuit_text: str, out_bits: str, **opts) -> "Program":
        return cls(sim_compile(circuit_text, amplitude_query(out_bits), **opts))

    @classmethod
    def compile_marginal(cls, circuit_text: str, n_qubits: int, qubit: int, value: int, **opts) -> "Program":
        return cls(sim_compile(circuit_text, marginal_query(n_qubits, qubit, value), **opts))

    def info(self) -> dict:
        return sim_program_info(self.handle)

    def ir(self) -> str:
        return sim_program_ir(self.handle)

    def layout(self):
        return sim_program_layout(self.handle)

    def evaluate(self, stream=None):
        return sim_eval_amplitude(self.handle, stream)

    def evaluate_range(self, first_slice: int, n_slices: int, stream=None):
        return sim_eval_range(self.handle, first_slice, n_slices, stream)

    def finalize(self, raw, stream=None):
        return sim_finalize(self.handle, raw, stream)

    def free(self):
        if self.handle:
            sim_program_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def evaluate_batch(programs, stream=None, tuning=None):
    return sim_eval_batch([p.handle for p in programs], stream, tuning)
