"""Compiled circuits evaluated on the GPU through the C-ABI, against the oracle (needs an
MI355X): exact state vector for small circuits, term-by-term evaluator for larger ones."""

import sys

import pytest

import paper_2403_06777_amd as zx
import workloads as wl
from oracle import statevector as sv

pytestmark = pytest.mark.gpu


def say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def gpu_compiled(text, query, **kw):
    h = zx.sim_compile(text, query, **kw)
    try:
        return zx.sim_eval_amplitude(h), zx.sim_program_info(h)
    finally:
        zx.sim_program_free(h)


def test_tiny_configuration_on_gpu():
    for seed in range(100):
        c, y = wl.tiny_circuit(seed)
        text = wl.circuit_text(c)
        got, _ = gpu_compiled(text, zx.amplitude_query(y))
        assert got == sv.exact_amplitude(text, y), seed


def test_marginals_on_gpu():
    for seed in range(20):
        rng = wl.SplitMix64(710, seed)
        n = 3 + seed % 6
        c = wl.random_clifford_t(rng, n, 40 + 5 * seed, 2 + seed % 7)
        text = wl.circuit_text(c)
        q = seed % n
        for v in (0, 1):
            got, _ = gpu_compiled(text, zx.marginal_query(n, q, v))
            assert got == sv.exact_marginal(text, q, v)


@pytest.mark.parametrize("seed", range(3))
def test_circuit_scale_exact(o2, seed):
    c, y = wl.circuit_scale(seed)
    text = wl.circuit_text(c)
    ir, info = zx.sim_compile_to_ir(text, zx.amplitude_query(y))
    say("circuit scale", seed, info["n_params"])
    got, _ = gpu_compiled(text, zx.amplitude_query(y))
    assert got == o2.evaluate(ir)["canonical"]


def test_batch_queries_subset(o2):
    qs = wl.batch_queries(64)
    hs, irs = [], []
    try:
        for c, y in qs:
            text = wl.circuit_text(c)
            q = zx.amplitude_query(y)
            hs.append(zx.sim_compile(text, q))
            irs.append(zx.sim_compile_to_ir(text, q)[0])
        single = [zx.sim_eval_amplitude(h) for h in hs]
        say("batch of", len(hs))
        assert zx.sim_eval_batch(hs) == single
        for h, ir, s in zip(hs, irs, single):
            if zx.sim_program_info(h)["n_params"] <= 22:
                assert s == o2.evaluate(ir)["canonical"]
    finally:
        for h in hs:
            zx.sim_program_free(h)


def _strings(n):
    return ["".join("1" if idx >> i & 1 else "0" for i in range(n)) for idx in range(1 << n)]


def test_outcome_parametric_all_strings_on_gpu():
    # one compilation per circuit; every output string's amplitude from one batched call
    from oracle import zomega as zw
    for seed in range(10):
        c, _ = wl.tiny_circuit(seed)
        text = wl.circuit_text(c)
        h = zx.sim_compile(text, zx.outcomes_query(c.n_qubits))
        try:
            ys = _strings(c.n_qubits)
            say("outcomes tiny", seed, zx.sim_program_info(h)["n_params"])
            got = zx.sim_eval_outcomes(h, ys)
            st = sv.exact_state(text)
            assert got == [zw.canonical(st.vec[i], -st.k) for i in range(len(ys))], seed
            # a repeated call on a subset equals the first
            assert zx.sim_eval_outcomes(h, ys[5:9]) == got[5:9]
        finally:
            zx.sim_program_free(h)


def test_outcome_parametric_matches_per_string_compilation():
    # larger circuits: sampled strings against compiling each string on its own
    for seed in range(4):
        rng = wl.SplitMix64(720, seed)
        n = 10 + 2 * seed
        c = wl.random_clifford_t(rng, n, 150 + 40 * seed, 10 + 2 * seed)
        text = wl.circuit_text(c)
        h = zx.sim_compile(text, zx.outcomes_query(n), p_cap=40)
        try:
            info = zx.sim_program_info(h)
            ys = ["".join("1" if rng.bernoulli(0.5) else "0" for _ in range(n)) for _ in range(12)]
            say("outcomes vs per-string", seed, n, info["n_params"], info["n_outer"])
            got = zx.sim_eval_outcomes(h, ys)
            for y, g in zip(ys, got):
                assert g == gpu_compiled(text, zx.amplitude_query(y), p_cap=40)[0], (seed, y)
        finally:
            zx.sim_program_free(h)


def test_outcome_parametric_rejects_plain_programs():
    c, y = wl.tiny_circuit(1)
    h = zx.sim_compile(wl.circuit_text(c), zx.amplitude_query(y))
    try:
        with pytest.raises(zx.SimError):
            zx.sim_eval_outcomes(h, [y])
    finally:
        zx.sim_program_free(h)
