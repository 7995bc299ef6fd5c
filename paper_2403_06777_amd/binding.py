"""ctypes binding of libzxpar.so: argument marshalling only.

Every function here has the name of the C entry point it calls and does nothing but convert
Python values to C arguments and back; all evaluation happens in the library's HIP kernels.
The library is loaded from this package directory; if it has not been built, importing a
function raises instead of falling back to anything else.

Scalars are returned as ``((c0, c1, c2, c3), e)`` meaning (c0 + c1 w + c2 w^2 + c3 w^3) *
sqrt2^e with w = e^{i pi/4}; raw partial sums as ``(c0, c1, c2, c3)``.
"""

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzxpar.so")

SIM_OK = 0
SIM_EINVAL = -1
SIM_ERANGE = -2
SIM_ENOMEM = -3
SIM_EDEVICE = -4
SIM_EBUSY = -5
SIM_ZOMEGA_RAW = 1
SIM_QUERY_AMPLITUDE = 0
SIM_QUERY_MARGINAL = 1
SIM_QUERY_OUTCOMES = 2
SIM_QUERY_PREFIX = 3

_CODES = {SIM_EINVAL: "SIM_EINVAL", SIM_ERANGE: "SIM_ERANGE", SIM_ENOMEM: "SIM_ENOMEM",
          SIM_EDEVICE: "SIM_EDEVICE", SIM_EBUSY: "SIM_EBUSY"}


class SimError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_CODES.get(code, code)}: {message}")
        self.code = code


class sim_i128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_int64)]

    def value(self) -> int:
        return (self.hi << 64) | self.lo

    @classmethod
    def of(cls, v: int) -> "sim_i128":
        if not -(1 << 127) <= v < (1 << 127):
            raise OverflowError("value does not fit int128")
        return cls(v & ((1 << 64) - 1), v >> 64)


class sim_zomega(ctypes.Structure):
    _fields_ = [("c", sim_i128 * 4), ("sqrt2_exp", ctypes.c_int32), ("flags", ctypes.c_uint32)]

    def coeffs(self) -> Tuple[int, int, int, int]:
        return tuple(self.c[k].value() for k in range(4))


class sim_query(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("n_qubits", ctypes.c_uint32),
                ("out_bits", ctypes.POINTER(ctypes.c_uint8)), ("qubit", ctypes.c_uint32),
                ("value", ctypes.c_uint32)]


class sim_compile_opts(ctypes.Structure):
    _fields_ = [("p_cap", ctypes.c_uint32), ("eliminate_constraints", ctypes.c_uint32),
                ("t_spiders_only", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 5)]


class sim_info(ctypes.Structure):
    _fields_ = [("n_params", ctypes.c_uint32), ("n_forms", ctypes.c_uint32),
                ("n_factors", ctypes.c_uint32), ("n_monomials", ctypes.c_uint32),
                ("sqrt2_exp", ctypes.c_int32), ("walk_bits", ctypes.c_uint32),
                ("n_slices", ctypes.c_uint64), ("image_bytes", ctypes.c_uint64),
                ("log2_terms", ctypes.c_double), ("n_eval_params", ctypes.c_uint32),
                ("is_zero", ctypes.c_uint32), ("compile_seconds", ctypes.c_double),
                ("t_count", ctypes.c_uint32), ("n_constraints", ctypes.c_uint32),
                ("ops_per_term", ctypes.c_double), ("nonzero_fraction", ctypes.c_double),
                ("n_outer", ctypes.c_uint32), ("vanish_table_bits", ctypes.c_uint32),
                ("n_params_given", ctypes.c_uint32), ("n_eliminated", ctypes.c_uint32),
                ("n_form_monomials", ctypes.c_uint32), ("n_mono_forms", ctypes.c_uint32),
                ("block_sum32", ctypes.c_uint32), ("team_waves", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class sim_tuning(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("walk_bits", ctypes.c_uint32), ("chunk_log2", ctypes.c_uint32)]


_P = ctypes.c_void_p
_lib = None

# (name, restype, argtypes) of every entry point in include/zxpar.h
SIGNATURES = [
    ("sim_init", ctypes.c_int, [ctypes.c_int]),
    ("sim_program_from_ir", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_P)]),
    ("sim_program_from_ir_flags", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_uint32,
                                                 ctypes.POINTER(_P)]),
    ("sim_ir_info_flags", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_uint32,
                                         ctypes.POINTER(sim_info)]),
    ("sim_compile", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(sim_query),
                                   ctypes.POINTER(sim_compile_opts), ctypes.POINTER(_P)]),
    ("sim_program_info", ctypes.c_int, [_P, ctypes.POINTER(sim_info)]),
    ("sim_ir_info", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(sim_info)]),
    ("sim_compile_to_ir", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(sim_query),
                                         ctypes.POINTER(sim_compile_opts), ctypes.c_char_p, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(sim_info)]),
    ("sim_program_ir", ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    ("sim_program_layout", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32]),
    ("sim_ir_affine_layout", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64),
                                            ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32,
                                            ctypes.POINTER(ctypes.c_uint32)]),
    ("sim_program_affine_layout", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64),
                                                 ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32]),
    ("sim_eval_amplitude", ctypes.c_int, [_P, _P, ctypes.POINTER(sim_zomega)]),
    ("sim_eval_timed", ctypes.c_int, [_P, _P, ctypes.POINTER(sim_zomega), ctypes.POINTER(ctypes.c_float)]),
    ("sim_eval_range", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint64, _P, ctypes.POINTER(sim_zomega)]),
    ("sim_finalize", ctypes.c_int, [_P, ctypes.POINTER(sim_zomega), _P, ctypes.POINTER(sim_zomega)]),
    ("sim_eval_batch", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, _P, ctypes.POINTER(sim_tuning),
                                      ctypes.POINTER(sim_zomega)]),
    ("sim_batch_plan_create", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.POINTER(sim_tuning), _P,
                                             ctypes.POINTER(_P)]),
    ("sim_batch_plan_run", ctypes.c_int, [_P, _P, ctypes.POINTER(sim_zomega)]),
    ("sim_batch_plan_free", None, [_P]),
    ("sim_eval_outcomes", ctypes.c_int, [_P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint8), _P,
                                         ctypes.POINTER(sim_tuning), ctypes.POINTER(sim_zomega)]),
    ("sim_enqueue_amplitude", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("sim_marginal_sum", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint8), _P, ctypes.POINTER(sim_tuning),
                                        ctypes.POINTER(sim_zomega)]),
    ("sim_sample", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.c_size_t,
                                  ctypes.POINTER(ctypes.c_uint64), _P, ctypes.POINTER(sim_tuning),
                                  ctypes.POINTER(ctypes.c_uint8),
                                  ctypes.POINTER(sim_zomega)]),
    ("sim_eval_ranges", ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t, _P,
                                       ctypes.POINTER(sim_tuning), ctypes.POINTER(sim_zomega)]),
    ("sim_serve_step", ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(sim_zomega),
                                      ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t, _P,
                                      ctypes.POINTER(sim_tuning), ctypes.POINTER(sim_zomega)]),
    ("sim_serve_enqueue", ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t, _P, ctypes.c_size_t, _P,
                                         ctypes.POINTER(sim_tuning), _P]),
    ("sim_eval_ranges_static", ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_uint64),
                                              ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t, _P,
                                              ctypes.POINTER(sim_tuning), ctypes.POINTER(sim_zomega)]),
    ("sim_finalize_batch", ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(sim_zomega), ctypes.c_size_t, _P,
                                          ctypes.POINTER(sim_zomega)]),
    ("sim_raw_add", ctypes.c_int, [ctypes.POINTER(sim_zomega), ctypes.POINTER(sim_zomega),
                                   ctypes.POINTER(sim_zomega)]),
    ("sim_scratch_bytes", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.POINTER(sim_tuning),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    ("sim_eval_amplitude_ws", ctypes.c_int, [_P, _P, _P, ctypes.c_size_t, ctypes.POINTER(sim_zomega)]),
    ("sim_eval_range_ws", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _P, _P,
                                         ctypes.c_size_t, ctypes.POINTER(sim_zomega)]),
    ("sim_eval_batch_ws", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, _P, _P, ctypes.c_size_t,
                                         ctypes.POINTER(sim_tuning), ctypes.POINTER(sim_zomega)]),
    ("sim_batch_prepare", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.POINTER(sim_tuning), _P,
                                         ctypes.c_size_t, _P]),
    ("sim_enqueue_batch", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, _P, _P, ctypes.c_size_t,
                                         ctypes.POINTER(sim_tuning), _P]),
    ("sim_batch_forget", ctypes.c_int, [_P]),
    ("sim_program_free", None, [_P]),
    ("sim_last_error", ctypes.c_char_p, []),
    ("sim_device_cus", ctypes.c_int, []),
]


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # PyTorch ships its own HIP runtime with the same soname; loading it first makes the
        # library bind to that one runtime, so torch streams and devices are shared with it
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SIM_OK:
        raise SimError(rc, lib().sim_last_error().decode(errors="replace"))


def _stream(stream) -> Optional[int]:
    """hipStream_t from None (null stream), an int handle or a torch stream"""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    handle = getattr(stream, "cuda_stream", None)
    if handle is None:
        raise TypeError("stream must be None, an int handle or a torch.cuda.Stream")
    return handle


def _scalar(z: sim_zomega):
    return z.coeffs(), z.sqrt2_exp


def _query(kind: int, n_qubits: int, out_bits: Optional[Sequence[int]] = None, qubit: int = 0,
           value: int = 0):
    q = sim_query()
    q.kind = kind
    q.n_qubits = n_qubits
    keep = None
    if out_bits is not None:
        keep = (ctypes.c_uint8 * max(1, n_qubits))(*[int(b) for b in out_bits])
        q.out_bits = ctypes.cast(keep, ctypes.POINTER(ctypes.c_uint8))
    q.qubit = qubit
    q.value = value
    return q, keep


def amplitude_query(out_bits: str):
    return _query(SIM_QUERY_AMPLITUDE, len(out_bits), [1 if ch == "1" else 0 for ch in out_bits])


def marginal_query(n_qubits: int, qubit: int, value: int):
    return _query(SIM_QUERY_MARGINAL, n_qubits, None, qubit, value)


def outcomes_query(n_qubits: int):
    """Every output bit a parameter: one compilation for all output strings."""
    return _query(SIM_QUERY_OUTCOMES, n_qubits, None)


def prefix_query(n_qubits: int, k: int, prefix_bits: Optional[str] = None):
    """P(y_0 .. y_{k-1}) over the first k qubits: with the outcomes as parameters (default)
    or for the fixed string prefix_bits (k characters)."""
    bits = None
    if prefix_bits is not None:
        if len(prefix_bits) != k:
            raise ValueError("prefix_bits must have k characters")
        bits = [1 if ch == "1" else 0 for ch in prefix_bits]
    return _query(SIM_QUERY_PREFIX, n_qubits, bits, k)


def _opts(p_cap: int = 0, eliminate_constraints: bool = True, t_spiders_only: bool = False):
    o = sim_compile_opts()
    o.p_cap = p_cap
    o.eliminate_constraints = 1 if eliminate_constraints else 0
    o.t_spiders_only = 1 if t_spiders_only else 0
    return o


def _tuning(t: Optional[dict]):
    if not t:
        return None
    s = sim_tuning()
    for k, v in t.items():
        setattr(s, k, int(v))
    return ctypes.byref(s)


# ------------------------------------------------------------------ entry points

def sim_init(device: int = 0):
    _check(lib().sim_init(device))


def sim_program_from_ir(ir_text: str) -> int:
    data = ir_text.encode()
    h = _P()
    _check(lib().sim_program_from_ir(data, len(data), ctypes.byref(h)))
    return h.value


SIM_IR_KEEP_VANISHING = 1


def sim_program_from_ir_flags(ir_text: str, flags: int) -> int:
    data = ir_text.encode()
    h = _P()
    _check(lib().sim_program_from_ir_flags(data, len(data), flags, ctypes.byref(h)))
    return h.value


def sim_ir_info_flags(ir_text: str, flags: int) -> dict:
    data = ir_text.encode()
    out = sim_info()
    _check(lib().sim_ir_info_flags(data, len(data), flags, ctypes.byref(out)))
    return out.as_dict()


def sim_compile(circuit_text: str, query, p_cap: int = 0, eliminate_constraints: bool = True,
                t_spiders_only: bool = False) -> int:
    q, _keep = query
    data = circuit_text.encode()
    h = _P()
    o = _opts(p_cap, eliminate_constraints, t_spiders_only)
    _check(lib().sim_compile(data, len(data), ctypes.byref(q), ctypes.byref(o), ctypes.byref(h)))
    return h.value


def sim_program_info(prog: int) -> dict:
    out = sim_info()
    _check(lib().sim_program_info(prog, ctypes.byref(out)))
    return out.as_dict()


def sim_ir_info(ir_text: str) -> dict:
    data = ir_text.encode()
    out = sim_info()
    _check(lib().sim_ir_info(data, len(data), ctypes.byref(out)))
    return out.as_dict()


def sim_compile_to_ir(circuit_text: str, query, p_cap: int = 0, eliminate_constraints: bool = True,
                      t_spiders_only: bool = False):
    q, _keep = query
    data = circuit_text.encode()
    o = _opts(p_cap, eliminate_constraints, t_spiders_only)
    n = ctypes.c_size_t()
    info = sim_info()
    _check(lib().sim_compile_to_ir(data, len(data), ctypes.byref(q), ctypes.byref(o), None, 0,
                                   ctypes.byref(n), ctypes.byref(info)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().sim_compile_to_ir(data, len(data), ctypes.byref(q), ctypes.byref(o), buf, n.value + 1,
                                   ctypes.byref(n), None))
    return buf.value.decode(), info.as_dict()


def sim_program_ir(prog: int) -> str:
    n = ctypes.c_size_t()
    _check(lib().sim_program_ir(prog, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().sim_program_ir(prog, buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def sim_program_layout(prog: int) -> List[int]:
    p = sim_program_info(prog)["n_params"]
    arr = (ctypes.c_int32 * max(1, p))()
    _check(lib().sim_program_layout(prog, arr, p))
    return list(arr[:p])


def sim_ir_affine_layout(ir_text: str):
    """host only: (x0, cols) of the program the IR text packs to"""
    data = ir_text.encode()
    x0 = ctypes.c_uint64()
    p = ctypes.c_uint32()
    cols = (ctypes.c_uint64 * 64)()
    _check(lib().sim_ir_affine_layout(data, len(data), ctypes.byref(x0), cols, 64, ctypes.byref(p)))
    return x0.value, list(cols[:p.value])


def sim_program_affine_layout(prog: int):
    """(x0, cols): slice-ordered index t is the assignment x0 ^ xor of cols[j] over the bits j of t"""
    p = sim_program_info(prog)["n_params"]
    x0 = ctypes.c_uint64()
    cols = (ctypes.c_uint64 * max(1, p))()
    _check(lib().sim_program_affine_layout(prog, ctypes.byref(x0), cols, p))
    return x0.value, list(cols[:p])


def sim_eval_amplitude(prog: int, stream=None):
    out = sim_zomega()
    _check(lib().sim_eval_amplitude(prog, _stream(stream), ctypes.byref(out)))
    return _scalar(out)


def sim_eval_timed(prog: int, stream=None):
    """returns (scalar, kernel_ms)"""
    out = sim_zomega()
    ms = ctypes.c_float()
    _check(lib().sim_eval_timed(prog, _stream(stream), ctypes.byref(out), ctypes.byref(ms)))
    return _scalar(out), ms.value


def sim_eval_range(prog: int, first_slice: int, n_slices: int, stream=None):
    out = sim_zomega()
    _check(lib().sim_eval_range(prog, first_slice, n_slices, _stream(stream), ctypes.byref(out)))
    return out.coeffs()


def _raw(coeffs) -> sim_zomega:
    z = sim_zomega()
    for k in range(4):
        z.c[k] = sim_i128.of(int(coeffs[k]))
    z.flags = SIM_ZOMEGA_RAW
    return z


def sim_finalize(prog: int, raw_coeffs, stream=None):
    raw = _raw(raw_coeffs)
    out = sim_zomega()
    _check(lib().sim_finalize(prog, ctypes.byref(raw), _stream(stream), ctypes.byref(out)))
    return _scalar(out)


def sim_finalize_batch(progs: Sequence[int], raws, stream=None):
    n = len(progs)
    zs = (sim_zomega * max(1, n))(*[_raw(r) for r in raws])
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_finalize_batch(_prog_array(progs), zs, n, _stream(stream), outs))
    return [_scalar(outs[i]) for i in range(n)]


def sim_raw_add(a, b):
    za, zb, out = _raw(a), _raw(b), sim_zomega()
    _check(lib().sim_raw_add(ctypes.byref(za), ctypes.byref(zb), ctypes.byref(out)))
    return out.coeffs()


def _prog_array(progs):
    return (_P * max(1, len(progs)))(*progs)


def sim_eval_batch(progs: Sequence[int], stream=None, tuning: Optional[dict] = None):
    n = len(progs)
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_eval_batch(_prog_array(progs), n, _stream(stream), _tuning(tuning), outs))
    return [_scalar(outs[i]) for i in range(n)]


def sim_eval_ranges(progs: Sequence[int], first_slices: Sequence[int], n_slices: Sequence[int], stream=None,
                    tuning: Optional[dict] = None):
    n = len(progs)
    firsts = (ctypes.c_uint64 * max(1, n))(*first_slices)
    counts = (ctypes.c_uint64 * max(1, n))(*n_slices)
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_eval_ranges(_prog_array(progs), firsts, counts, n, _stream(stream), _tuning(tuning), outs))
    return [outs[i].coeffs() for i in range(n)]


def sim_serve_step(progs: Sequence[int], first_slices: Sequence[int], n_slices: Sequence[int], carries,
                   last: Sequence[bool], stream=None, tuning: Optional[dict] = None):
    """One continuous-batching step: entry i is the raw sum (coefficients) of its slices plus
    carries[i] when last[i] is false, else the finalised ((coefficients), e)."""
    n = len(progs)
    firsts = (ctypes.c_uint64 * max(1, n))(*first_slices)
    counts = (ctypes.c_uint64 * max(1, n))(*n_slices)
    cz = (sim_zomega * max(1, n))(*[_raw(c) for c in carries])
    lz = (ctypes.c_uint8 * max(1, n))(*[1 if x else 0 for x in last])
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_serve_step(_prog_array(progs), firsts, counts, cz, lz, n, _stream(stream), _tuning(tuning),
                                outs))
    return [_scalar(outs[i]) if last[i] else outs[i].coeffs() for i in range(n)]


def sim_serve_enqueue(progs: Sequence[int], first_slices: Sequence[int], n_slices: Sequence[int],
                      slots: Sequence[int], flags: Sequence[int], dev_carry: int, n_carry_slots: int, dev_out: int,
                      stream=None, tuning: Optional[dict] = None):
    """Enqueues one pipelined serving step (device-resident carried sums; see zxpar.h)."""
    n = len(progs)
    firsts = (ctypes.c_uint64 * max(1, n))(*first_slices)
    counts = (ctypes.c_uint64 * max(1, n))(*n_slices)
    sl = (ctypes.c_uint32 * max(1, n))(*slots)
    fl = (ctypes.c_uint8 * max(1, n))(*flags)
    _check(lib().sim_serve_enqueue(_prog_array(progs), firsts, counts, sl, fl, n, dev_carry, n_carry_slots,
                                   _stream(stream), _tuning(tuning), dev_out))


def sim_eval_ranges_static(progs: Sequence[int], first_slices: Sequence[int], n_slices: Sequence[int],
                           stream=None, tuning: Optional[dict] = None):
    """sim_eval_ranges in the library's fixed 4 MiB device array (no allocation)"""
    n = len(progs)
    firsts = (ctypes.c_uint64 * max(1, n))(*first_slices)
    counts = (ctypes.c_uint64 * max(1, n))(*n_slices)
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_eval_ranges_static(_prog_array(progs), firsts, counts, n, _stream(stream), _tuning(tuning),
                                        outs))
    return [outs[i].coeffs() for i in range(n)]


def sim_eval_outcomes(prog: int, out_strings: Sequence[str], stream=None, tuning: Optional[dict] = None):
    """Amplitudes <y|C|0> of an OUTCOMES program for output strings such as "0110"."""
    n = len(out_strings)
    k = len(out_strings[0]) if n else 0
    bits = (ctypes.c_uint8 * max(1, n * k))(*[1 if ch == "1" else 0 for y in out_strings for ch in y])
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_eval_outcomes(prog, n, bits, _stream(stream), _tuning(tuning), outs))
    return [_scalar(outs[i]) for i in range(n)]


def sim_enqueue_amplitude(prog: int, dev_out: int, stream=None, ev_before: int = 0, ev_after: int = 0):
    """Enqueues an evaluation whose canonical value the device writes to dev_out (the address of
    72 bytes of device memory, 8-byte aligned); events (raw handles, 0 = none) bracket the kernel."""
    _check(lib().sim_enqueue_amplitude(prog, _stream(stream), ev_before or None, ev_after or None, dev_out))


def zomega_from_bytes(b: bytes):
    """(coefficients, sqrt2 exponent) of a 72-byte sim_zomega written by the device; raises on the
    overflow flag."""
    z = sim_zomega.from_buffer_copy(bytes(b))
    if z.flags & 2:
        raise SimError(-2, "int128 overflow while applying the program constant")
    return _scalar(z)


def sim_marginal_sum(prog: int, pattern: str, stream=None, tuning: Optional[dict] = None):
    """Sum of |amplitude|^2 over the output strings matching pattern ('0', '1' fixed, '*'
    free) of an OUTCOMES program."""
    code = {"0": 0, "1": 1, "*": 2}
    bits = (ctypes.c_uint8 * max(1, len(pattern)))(*[code[ch] for ch in pattern])
    out = sim_zomega()
    _check(lib().sim_marginal_sum(prog, bits, _stream(stream), _tuning(tuning), ctypes.byref(out)))
    return _scalar(out)


def sim_sample(progs: Sequence[int], uniforms, stream=None, tuning: Optional[dict] = None):
    """Repeated weak simulation: progs[k-1] is the prefix program of the first k qubits
    (k = 1 .. K), uniforms an (n, K) array of 53-bit integers.  Returns the (n, K) uint8 array
    of sampled bits and each sample's probability as (coefficients, sqrt2 exponent)."""
    import numpy as np
    u = np.ascontiguousarray(uniforms, dtype=np.uint64)
    if u.ndim != 2 or u.shape[1] != len(progs):
        raise ValueError("uniforms must be an (n, K) array with K = len(progs)")
    n, K = u.shape
    bits = np.zeros((n, K), dtype=np.uint8)
    probs = (sim_zomega * max(1, n))()
    _check(lib().sim_sample(_prog_array(progs), K, n, u.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                            _stream(stream), _tuning(tuning), bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            probs))
    return bits, [_scalar(probs[i]) for i in range(n)]


def sim_batch_plan_create(progs: Sequence[int], tuning: Optional[dict] = None, stream=None) -> int:
    h = _P()
    _check(lib().sim_batch_plan_create(_prog_array(progs), len(progs), _tuning(tuning), _stream(stream),
                                       ctypes.byref(h)))
    return h.value


def sim_batch_plan_run(plan: int, n: int, stream=None):
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_batch_plan_run(plan, _stream(stream), outs))
    return [_scalar(outs[i]) for i in range(n)]


def sim_batch_plan_free(plan: int):
    lib().sim_batch_plan_free(plan)


def sim_scratch_bytes(progs: Sequence[int], tuning: Optional[dict] = None) -> int:
    """bytes of caller-owned device scratch the *_ws calls and sim_enqueue_batch need"""
    out = ctypes.c_size_t()
    _check(lib().sim_scratch_bytes(_prog_array(progs), len(progs), _tuning(tuning), ctypes.byref(out)))
    return out.value


def sim_eval_amplitude_ws(prog: int, dev_scratch: int, scratch_bytes: int, stream=None):
    out = sim_zomega()
    _check(lib().sim_eval_amplitude_ws(prog, _stream(stream), dev_scratch, scratch_bytes, ctypes.byref(out)))
    return _scalar(out)


def sim_eval_range_ws(prog: int, first: int, count: int, g: int, dev_scratch: int, scratch_bytes: int,
                      stream=None):
    out = sim_zomega()
    _check(lib().sim_eval_range_ws(prog, first, count, g, _stream(stream), dev_scratch, scratch_bytes,
                                   ctypes.byref(out)))
    return out.coeffs()


def sim_eval_batch_ws(progs: Sequence[int], dev_scratch: int, scratch_bytes: int, stream=None,
                      tuning: Optional[dict] = None):
    n = len(progs)
    outs = (sim_zomega * max(1, n))()
    _check(lib().sim_eval_batch_ws(_prog_array(progs), n, _stream(stream), dev_scratch, scratch_bytes,
                                   _tuning(tuning), outs))
    return [_scalar(outs[i]) for i in range(n)]


def sim_batch_prepare(progs: Sequence[int], dev_scratch: int, scratch_bytes: int, stream=None,
                      tuning: Optional[dict] = None):
    _check(lib().sim_batch_prepare(_prog_array(progs), len(progs), _tuning(tuning), dev_scratch, scratch_bytes,
                                   _stream(stream)))


def sim_enqueue_batch(progs: Sequence[int], dev_scratch: int, scratch_bytes: int, dev_out: int, stream=None,
                      tuning: Optional[dict] = None):
    """Enqueues a prepared batch; the device writes len(progs) 72-byte results to dev_out."""
    _check(lib().sim_enqueue_batch(_prog_array(progs), len(progs), _stream(stream), dev_scratch, scratch_bytes,
                                   _tuning(tuning), dev_out))


def sim_batch_forget(dev_scratch: int):
    _check(lib().sim_batch_forget(dev_scratch))


def zomegas_from_bytes(b: bytes, n: int):
    """n results of 72 bytes each, as written by the device (sim_enqueue_batch)"""
    return [zomega_from_bytes(bytes(b[72 * i:72 * (i + 1)])) for i in range(n)]


def sim_program_free(prog: int):
    lib().sim_program_free(prog)


def sim_last_error() -> str:
    return lib().sim_last_error().decode(errors="replace")


def sim_device_cus() -> int:
    return lib().sim_device_cus()
