"""Prefix marginals and repeated weak simulation on the GPU through the C-ABI (needs an
MI355X): prefix programs against the exact state vector, samples against the chain-rule
oracle on the same uniforms."""

import sys

import numpy as np
import pytest

import paper_2403_06777_amd as zx
import workloads as wl
from oracle import sampling as osamp
from oracle import statevector as sv

pytestmark = pytest.mark.gpu


def say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def compile_prefixes(text, n, K, **kw):
    return [zx.sim_compile(text, zx.prefix_query(n, k), **kw) for k in range(1, K + 1)]


def free_all(hs):
    for h in hs:
        zx.sim_program_free(h)


def _bits(idx, k):
    return "".join("1" if idx >> i & 1 else "0" for i in range(k))


def test_prefix_programs_on_gpu():
    for seed in range(6):
        c, _ = wl.tiny_circuit(seed)
        text = wl.circuit_text(c)
        n = c.n_qubits
        hs = compile_prefixes(text, n, n)
        try:
            for k, h in enumerate(hs, start=1):
                say("prefix programs", seed, k, zx.sim_program_info(h)["n_params"])
                pres = [_bits(i, k) for i in range(1 << k)]
                got = zx.sim_eval_outcomes(h, pres)
                assert got == [sv.exact_prefix_marginal(text, b) for b in pres], (seed, k)
        finally:
            free_all(hs)


@pytest.mark.parametrize("seed", range(6))
def test_samples_match_the_oracle(seed):
    c, _ = wl.tiny_circuit(seed)
    text = wl.circuit_text(c)
    n = c.n_qubits
    u = wl.sampling_uniforms(seed, 400, n)
    hs = compile_prefixes(text, n, n)
    try:
        say("sample tiny", seed)
        bits, probs = zx.sim_sample(hs, u)
        want, wprobs = osamp.weak_samples(text, u.tolist())
        assert ["".join(str(b) for b in row) for row in bits] == want
        assert probs == wprobs
        # the same uniforms give the same samples
        again, _ = zx.sim_sample(hs, u[:37])
        assert np.array_equal(again, bits[:37])
    finally:
        free_all(hs)


@pytest.mark.parametrize("seed", range(4))
def test_samples_random_circuits_and_partial_prefixes(seed):
    rng = wl.SplitMix64(730, seed)
    n = 8 + seed
    c = wl.random_clifford_t(rng, n, 100 + 30 * seed, 8 + 3 * seed)
    text = wl.circuit_text(c)
    K = n if seed % 2 == 0 else 3
    u = wl.sampling_uniforms(100 + seed, 300, K)
    hs = compile_prefixes(text, n, K)
    try:
        say("sample random", seed, n, K, [zx.sim_program_info(h)["n_params"] for h in hs])
        bits, probs = zx.sim_sample(hs, u)
        want, wprobs = osamp.weak_samples(text, u.tolist(), K)
        assert ["".join(str(b) for b in row) for row in bits] == want
        assert probs == wprobs
    finally:
        free_all(hs)


def test_samples_at_full_size_against_the_complex_state():
    # 20 qubits, 400 Clifford + 32 T: every decision whose margin exceeds the rounding of a
    # complex128 state vector is checked, and each sample's exact probability is its |amp|^2
    from oracle import zomega as zw
    c = wl.sampling_circuit(0)
    text = wl.circuit_text(c)
    n = c.n_qubits
    N = 64
    u = wl.sampling_uniforms(7, N, n)
    hs = compile_prefixes(text, n, n, p_cap=40)
    try:
        say("sample full size", [zx.sim_program_info(h)["n_params"] for h in hs])
        bits, probs = zx.sim_sample(hs, u)
    finally:
        free_all(hs)
    p = np.abs(sv.complex_state(text)) ** 2
    marg = [p.reshape(-1, 1 << k).sum(axis=0) for k in range(n + 1)]  # marg[k][prefix]
    checked = 0
    for i in range(N):
        prefix = 0
        for k in range(n):
            cond = marg[k + 1][prefix] / marg[k][prefix]
            x = float(u[i, k]) / 2.0 ** 53
            if abs(x - cond) > 1e-9:
                assert bits[i, k] == (0 if x < cond else 1), (i, k)
                checked += 1
            prefix |= int(bits[i, k]) << k
        assert abs(zw.to_complex(*probs[i]) - p[prefix]) <= 1e-9 * p[prefix] + 1e-15
    assert checked >= N * n - 4


def test_sample_arguments_are_checked():
    c, _ = wl.tiny_circuit(0)
    text = wl.circuit_text(c)
    hs = compile_prefixes(text, 6, 2)
    odd = zx.sim_compile("qubits 1\nh 0\nt 0\nh 0\n", zx.outcomes_query(1))
    try:
        with pytest.raises(zx.SimError) as ei:
            zx.sim_sample([hs[1], hs[0]], wl.sampling_uniforms(0, 4, 2))
        assert ei.value.code == -1 and "query parameters" in str(ei.value)
        u = wl.sampling_uniforms(0, 4, 2)
        u[2, 1] = 1 << 53
        with pytest.raises(zx.SimError) as ei:
            zx.sim_sample(hs, u)
        assert "2^53" in str(ei.value)
        # an amplitude program is not a probability: <0|HTH|0> = (1 + w) / 2 is not real
        with pytest.raises(zx.SimError) as ei:
            zx.sim_sample([odd], wl.sampling_uniforms(0, 4, 1))
        assert "not real" in str(ei.value)
        bits, probs = zx.sim_sample(hs, np.zeros((0, 2), dtype=np.uint64))
        assert bits.shape == (0, 2) and probs == []
    finally:
        free_all(hs + [odd])
