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


def _random_pattern(rng, n):
    return "".join("*01"[rng.randint(0, 2)] for _ in range(n))


def test_marginals_by_summing_match_the_oracle():
    # Fig. 3 left: squares of the outcome-parametric amplitudes, summed exactly
    for seed in range(8):
        rng = wl.SplitMix64(740, seed)
        if seed < 4:
            c, _ = wl.tiny_circuit(seed)
        else:
            c = wl.random_clifford_t(rng, 4 + seed, 120 + 20 * seed, 10 + seed)
        text = wl.circuit_text(c)
        n = c.n_qubits
        h = zx.sim_compile(text, zx.outcomes_query(n), p_cap=40)
        try:
            say("marginal by summing", seed, n, zx.sim_program_info(h)["n_params"])
            assert zx.sim_marginal_sum(h, "*" * n) == ((1, 0, 0, 0), 0)
            pats = [_random_pattern(rng, n) for _ in range(6)] + ["1" + "*" * (n - 1), "0" * n]
            for pat in pats:
                assert zx.sim_marginal_sum(h, pat) == sv.exact_marginal_pattern(text, pat), (seed, pat)
        finally:
            zx.sim_program_free(h)


def test_summing_equals_doubling():
    # the two forms of a marginal (Fig. 3): summed squares of amplitudes and the doubled
    # diagram's prefix program give the same exact value
    for seed in range(4):
        rng = wl.SplitMix64(750, seed)
        n = 10
        c = wl.random_clifford_t(rng, n, 160, 14)
        text = wl.circuit_text(c)
        h = zx.sim_compile(text, zx.outcomes_query(n), p_cap=40)
        hp = zx.sim_compile(text, zx.prefix_query(n, 4), p_cap=40)
        try:
            for idx in range(16):
                pre = _bits(idx, 4)
                assert zx.sim_marginal_sum(h, pre + "*" * (n - 4)) == zx.sim_eval_outcomes(hp, [pre])[0]
        finally:
            zx.sim_program_free(h)
            zx.sim_program_free(hp)


def test_marginal_sum_arguments_are_checked():
    n = 34
    text = f"qubits {n}\n" + "".join(f"h {q}\n" for q in range(n)) + "t 0\nh 0\n"
    h = zx.sim_compile(text, zx.outcomes_query(n))
    c, _ = wl.tiny_circuit(0)
    plain = zx.sim_compile(wl.circuit_text(c), zx.amplitude_query("0" * 6))
    try:
        with pytest.raises(zx.SimError) as ei:
            zx.sim_marginal_sum(h, "*" * 33 + "0")
        assert ei.value.code == -2 and "32 summed" in str(ei.value)
        with pytest.raises(zx.SimError) as ei:
            zx.sim_marginal_sum(plain, "*" * 6)
        assert ei.value.code == -1
        # Qubit 0 is in HTH|0> = ((1 + w)|0> + (1 - w)|1>) / 2, the others in |+>:
        # P(y_0 = 0, y_23..32 = 0, y_33 = 1) = (2 + sqrt2) / 4 * 2^-11 = (1 + sqrt2) sqrt2^-25,
        # summed over 2^22 strings (64 batches of 2^16 amplitudes, squares added on the device);
        # with qubit 0 free and 16 qubits fixed it is 2^-16
        assert zx.sim_marginal_sum(h, "0" + "*" * 22 + "0" * 10 + "1") == ((1, 1, 0, -1), -25)
        assert zx.sim_marginal_sum(h, "*" * 18 + "1" * 16) == ((1, 0, 0, 0), -32)
    finally:
        zx.sim_program_free(h)
        zx.sim_program_free(plain)
