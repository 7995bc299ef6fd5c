"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: a value printed in or
derived from the paper, a closed form, an invariant of the sum, or a library routine.
"""

import cmath
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as wl
from oracle import statevector as sv
from oracle import zomega as zw
from workloads.programs import ProgramSpec

W = cmath.exp(1j * math.pi / 4)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit_forms(prog: ProgramSpec):
    return [prog.add_form(0, 1 << i) for i in range(prog.p)]


# ----------------------------------------------------------------- Z[w] arithmetic

def test_omega_powers_match_complex_exponential():
    # w^k is e^{i k pi/4} (the lookup table of Section 3.3 step 5), via the library exp
    for k in range(-9, 17):
        assert abs(zw.to_complex(zw.omega_pow(k)) - cmath.exp(1j * math.pi * k / 4)) < 1e-12


def test_product_matches_complex_multiplication():
    rng = wl.SplitMix64(900, 1)
    for _ in range(200):
        a = tuple(rng.randint(-50, 50) for _ in range(4))
        b = tuple(rng.randint(-50, 50) for _ in range(4))
        assert abs(zw.to_complex(zw.mul(a, b)) - zw.to_complex(a) * zw.to_complex(b)) < 1e-8


def _to_abcd(z):
    # the paper's coordinates A + B sqrt2 + i (C + D sqrt2)
    c0, c1, c2, c3 = z
    return (Fraction(c0), Fraction(c1 - c3, 2), Fraction(c2), Fraction(c1 + c3, 2))


def test_lemma6_lemma7_sum_and_product_in_paper_coordinates():
    # Appendix E, Lemmas 6 and 7: sums and products of A + B sqrt2 + i(C + D sqrt2)
    rng = wl.SplitMix64(901, 2)
    for _ in range(200):
        z1 = tuple(rng.randint(-30, 30) for _ in range(4))
        z2 = tuple(rng.randint(-30, 30) for _ in range(4))
        A1, B1, C1, D1 = _to_abcd(z1)
        A2, B2, C2, D2 = _to_abcd(z2)
        # Lemma 6
        assert _to_abcd(zw.add(z1, z2)) == (A1 + A2, B1 + B2, C1 + C2, D1 + D2)
        # Lemma 7
        A = A1 * A2 + 2 * B1 * B2 - C1 * C2 - 2 * D1 * D2
        B = A1 * B2 + B1 * A2 - C1 * D2 - D1 * C2
        C = A1 * C2 + 2 * B1 * D2 + C1 * A2 + 2 * D1 * B2
        D = A1 * D2 + B1 * C2 + C1 * B2 + D1 * A2
        assert _to_abcd(zw.mul(z1, z2)) == (A, B, C, D)


def test_canonical_form():
    # 2 = sqrt2^2, sqrt2 = w - w^3, 1 + i = sqrt2 w, and zero is ((0,0,0,0), 0)
    assert zw.canonical((2, 0, 0, 0), 0) == ((1, 0, 0, 0), 2)
    assert zw.canonical((0, 1, 0, -1), 0) == ((1, 0, 0, 0), 1)
    assert zw.canonical((1, 0, 1, 0), 0) == ((0, 1, 0, 0), 1)
    assert zw.canonical((0, 0, 0, 0), 7) == ((0, 0, 0, 0), 0)
    rng = wl.SplitMix64(902, 3)
    for _ in range(100):
        z = tuple(rng.randint(-40, 40) for _ in range(4))
        e = rng.randint(-5, 5)
        c, ce = zw.canonical(z, e)
        assert abs(zw.to_complex(c, ce) - zw.to_complex(z, e)) < 1e-9
        assert zw.canonical(zw.times_sqrt2(z), e - 1) == (c, ce)


# ----------------------------------------------------------------- term evaluator

def test_appendix_d_worked_example(o2):
    rows, values, total = [], {}, None
    with open(os.path.join(GOLDEN, "appendix_d.txt")) as f:
        for line in f:
            tok = line.split("#", 1)[0].split()
            if not tok:
                continue
            if tok[0] == "row":
                rows.append([int(v) for v in tok[1:]])
            elif tok[0] == "value":
                values[tok[1]] = tuple(int(v) for v in tok[2:])
            elif tok[0] == "total":
                total = tuple(int(v) for v in tok[1:])
    assert len(rows) == 6 and len(values) == 16

    def subterm(row, bits):
        flag, a, psi, b, phi = row[0], row[1], row[2:6], row[6], row[7:11]
        if not flag:
            return 1.0
        x = sum(p & q for p, q in zip(psi, bits)) % 2
        y = sum(p & q for p, q in zip(phi, bits)) % 2
        Psi = a * math.pi / 4 + math.pi * x
        Phi = b * math.pi / 4 + math.pi * y
        return 1 + cmath.exp(1j * Psi) + cmath.exp(1j * Phi) - cmath.exp(1j * (Psi + Phi))

    # the stored values agree with a direct complex evaluation of Eq. 3 on the table
    for key, val in values.items():
        bits = [int(ch) for ch in key]
        direct = np.prod([subterm(r, bits) for r in rows[0:3]]) + np.prod([subterm(r, bits) for r in rows[3:6]])
        assert abs(direct - zw.to_complex(val)) < 1e-9

    # the oracle on the two terms of the table reproduces every value and the total
    terms = wl.appendix_d_terms()
    per = [o2.evaluate(t.to_text(), terms=True, threads=1)["terms"] for t in terms]
    acc = zw.ZERO
    for key, val in values.items():
        x = sum(int(ch) << k for k, ch in enumerate(key))
        got = zw.add(per[0][x], per[1][x])
        assert got == val, key
        acc = zw.add(acc, got)
    assert acc == total == (80, 0, 16, 0)


@pytest.mark.parametrize("p", [1, 3, 6])
def test_node_pair_cancellation_identities(o2, p):
    # Section 5: (1 + e^{i pi (2/4 + l)}) (1 + e^{i pi (6/4 + l)}) = 2 for every parity l,
    # and the same with constants 0 and pi gives 0
    rng = wl.SplitMix64(903, p)
    prog = ProgramSpec(p)
    f = prog.add_form(rng.randint(0, 1), (1 << p) - 1)
    prog.nodes += [(f, 2, 4), (f, 6, 4)]
    assert o2.evaluate(prog.to_text())["raw"] == (2 * 2 ** p, 0, 0, 0)
    prog.nodes = [(f, 0, 4), (f, 4, 4)]
    assert o2.evaluate(prog.to_text())["raw"] == (0, 0, 0, 0)


def _terms(o2, prog):
    return o2.evaluate(prog.to_text(), terms=True, threads=1)["terms"]


@pytest.mark.parametrize("a", range(8))
def test_lemma4_pi_pair_is_half_a_phase_pair(o2, a):
    # Appendix C, Lemma 4: e^{i Psi Phi / pi} = (1/2)(1 + e^{i Psi} + e^{i Phi} - e^{i(Psi+Phi)})
    # when Phi is 0 or pi.  Psi = a pi/4 + pi x0, Phi = pi x1 so Psi Phi / pi in units of
    # pi/4 is (a + 4 x0) x1 = a x1 + 4 x0 x1.
    lhs = ProgramSpec(2)
    lhs.mono = [(a % 8, [1]), (4, [0, 1])] if a % 8 else [(4, [0, 1])]
    rhs = ProgramSpec(2)
    u = _unit_forms(rhs)
    rhs.pairs = [(u[0], u[1], a, 0)]
    tl, tr = _terms(o2, lhs), _terms(o2, rhs)
    for x in range(4):
        assert zw.scale(tl[x], 2) == tr[x]


@pytest.mark.parametrize("a", range(8))
def test_lemma3_node_as_phase_pair(o2, a):
    # Appendix C, Lemma 3 read with Phi = pi/2 and C = (1 - i)/2:
    # 1 + e^{i Psi} = C (1 + e^{i Psi'} + e^{i Phi} - e^{i(Psi' + Phi)}), Psi' = Psi + pi/2
    node = ProgramSpec(1)
    f = node.add_form(0, 1)
    node.nodes = [(f, a, 4)]
    pair = ProgramSpec(1)
    f1 = pair.add_form(0, 1)
    f0 = pair.add_form(0, 0)
    pair.pairs = [(f1, f0, a + 2, 2)]
    tn, tp = _terms(o2, node), _terms(o2, pair)
    one_minus_i = (1, 0, -1, 0)
    for x in range(2):
        assert zw.scale(tn[x], 2) == zw.mul(one_minus_i, tp[x])


def test_lemma5_half_pi_as_phase_pair(o2):
    # Appendix C, Lemma 5 with the parity taken as the integer 0/1: for Psi = pi/2 + pi x,
    # e^{i Psi / 2} = w * w^{2x}, and w^{2x} = (1/2)(1 + e^{i pi x} + i - i e^{i pi x}),
    # the phase pair with Psi' = pi x and Phi = pi/2
    half = ProgramSpec(1)
    half.mono = [(2, [0])]
    half.scalar = (0, 1, 0, 0)
    pair = ProgramSpec(1)
    f1 = pair.add_form(0, 1)
    f0 = pair.add_form(0, 0)
    pair.pairs = [(f1, f0, 0, 2)]
    th, tp = _terms(o2, half), _terms(o2, pair)
    for x in range(2):
        direct = cmath.exp(1j * (math.pi / 2 + math.pi * x) / 2)
        assert abs(zw.to_complex(zw.mul((0, 1, 0, 0), th[x])) - direct) < 1e-12
        assert zw.scale(th[x], 2) == tp[x]


@pytest.mark.parametrize("seed", range(4))
def test_separable_product_closed_form(o2, seed):
    # sum over x of prod_i (1 + w^{k_i x_i}) = prod_i (2 + (1 + w^{k_i})) = prod_i (3 + w^{k_i})
    rng = wl.SplitMix64(904, seed)
    p = 8
    prog = ProgramSpec(p)
    u = _unit_forms(prog)
    ks = [rng.randint(0, 7) for _ in range(p)]
    prog.nodes = [(u[i], 0, ks[i]) for i in range(p)]
    expect = zw.ONE
    cval = 1.0
    for k in ks:
        expect = zw.mul(expect, zw.add((3, 0, 0, 0), zw.omega_pow(k)))
        cval *= 3 + cmath.exp(1j * math.pi * k / 4)
    got = o2.evaluate(prog.to_text())["raw"]
    assert got == expect
    assert abs(zw.to_complex(got) - cval) < 1e-6 * abs(cval) + 1e-9


@pytest.mark.parametrize("p", [2, 6, 10])
def test_gauss_sums(o2, p):
    # sum_x (-1)^{x0 x1 + x2 x3 + ...} = 2^{p/2};  sum_x i^{|x|} = (1 + i)^p;
    # sum_x (-1)^{m.x} = 0 for m != 0
    prog = ProgramSpec(p)
    prog.mono = [(4, [2 * i, 2 * i + 1]) for i in range(p // 2)]
    assert o2.evaluate(prog.to_text())["raw"] == (2 ** (p // 2), 0, 0, 0)
    prog = ProgramSpec(p)
    prog.mono = [(2, [i]) for i in range(p)]
    expect = zw.ONE
    for _ in range(p):
        expect = zw.mul(expect, (1, 0, 1, 0))
    assert o2.evaluate(prog.to_text())["raw"] == expect
    prog = ProgramSpec(p)
    f = prog.add_form(0, (1 << p) - 1)
    prog.lin = [(4, f)]
    assert o2.evaluate(prog.to_text())["raw"] == (0, 0, 0, 0)


@pytest.mark.parametrize("seed,scramble,mono", [(0, True, 0), (1, True, 0), (2, False, 2), (3, False, 3)])
def test_block_product_and_affine_invariance(o2, seed, scramble, mono):
    # the sum over all assignments is the product of independent block sums, and is
    # unchanged by an invertible affine relabelling of the variables
    full, blocks = wl.block_separable_program(seed, 14, factors_per_block=3, lin_per_block=1,
                                              mono_per_block=mono, pairs_per_block=1 if scramble else 0,
                                              scramble=scramble)
    expect = zw.ONE
    for blk in blocks:
        expect = zw.mul(expect, o2.evaluate(blk.to_text(), threads=1)["raw"])
    assert o2.evaluate(full.to_text())["raw"] == expect


def test_range_split_and_enumeration_order(o2):
    prog = wl.random_program(5, 12, n_nodes=10, n_pairs=2, n_lin=3, n_mono=15)
    text = prog.to_text()
    whole = o2.evaluate(text)["raw"]
    acc = zw.ZERO
    for first in range(0, 4096, 1000):
        acc = zw.add(acc, o2.evaluate(text, first=first, count=min(1000, 4096 - first))["raw"])
    assert acc == whole
    perm = list(range(12))[::-1]
    assert o2.evaluate(text, perm=perm)["raw"] == whole


def test_scalar_and_exponent_are_applied(o2):
    prog = wl.random_program(6, 5, n_nodes=4, n_lin=2, scalar_range=3)
    out = o2.evaluate(prog.to_text())
    assert out["value"] == (zw.mul(prog.scalar, out["raw"]), prog.sqrt2_exp)


def test_random_programs_match_complex_evaluation(o2):
    # floating-point cross-check of the whole definition on small random programs
    for seed in range(6):
        prog = wl.random_program(seed, 6, n_nodes=6, n_pairs=2, n_lin=2, n_mono=6, scalar_range=2)
        total = 0
        for x in range(2 ** prog.p):
            lf = [(c ^ bin(m & x).count("1")) & 1 for c, m in prog.forms]
            t = 1
            for f, a, b in prog.nodes:
                t *= 1 + W ** (a + b * lf[f])
            for f1, f2, a, b in prog.pairs:
                l1, l2 = lf[f1], lf[f2]
                t *= 1 + W ** (a + 4 * l1) + W ** (b + 4 * l2) - W ** (a + b + 4 * (l1 ^ l2))
            ph = sum(c * lf[f] for c, f in prog.lin) + sum(c * all(x >> v & 1 for v in vs) for c, vs in prog.mono)
            total += t * W ** ph
        total *= zw.to_complex(prog.scalar, prog.sqrt2_exp)
        got = o2.evaluate(prog.to_text())["value"]
        assert abs(zw.to_complex(*got) - total) < 1e-7 * max(1, abs(total))


def test_overflow_is_reported(o2):
    # 2^70 * 2^? terms cannot be held: the oracle must refuse, not wrap
    prog = ProgramSpec(1)
    prog.scalar = (2 ** 100, 0, 0, 0)
    f = prog.add_form(0, 0)
    prog.nodes = [(f, 0, 0)] * 40
    with pytest.raises(o2.OracleOverflow):
        o2.evaluate(prog.to_text())


# ----------------------------------------------------------------- state vector

def _dense_unitary(n, gates):
    H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    mats = {"h": H, "x": np.array([[0, 1], [1, 0]])}
    for g, k in sv.DIAG_PHASE.items():
        mats[g] = np.diag([1, np.exp(1j * np.pi * k / 4)])
    U = np.eye(2 ** n, dtype=complex)
    for g in gates:
        if g[0] in mats:
            # qubit q is bit q of the basis index: kron order is qubit n-1 ... qubit 0
            ops = [np.eye(2)] * n
            ops[n - 1 - g[1]] = mats[g[0]]
            M = ops[0]
            for o in ops[1:]:
                M = np.kron(M, o)
        else:
            M = np.zeros((2 ** n, 2 ** n), dtype=complex)
            for i in range(2 ** n):
                if g[0] == "cx":
                    j = i ^ (1 << g[2]) if i >> g[1] & 1 else i
                    M[j, i] = 1
                else:
                    M[i, i] = -1 if (i >> g[1] & 1 and i >> g[2] & 1) else 1
        U = M @ U
    return U


@pytest.mark.parametrize("seed", range(5))
def test_statevector_matches_dense_unitary(seed):
    rng = wl.SplitMix64(905, seed)
    n = 4
    c = wl.random_clifford_t(rng, n, 30, 6)
    c.gates.insert(3, ("cz", 0, 2))
    c.gates.insert(7, ("x", 1))
    c.gates.insert(9, ("tdg", 3))
    c.gates.insert(11, ("sdg", 0))
    c.gates.insert(13, ("z", 2))
    text = wl.circuit_text(c)
    U = _dense_unitary(n, c.gates)
    st = sv.exact_state(text)
    for i in range(2 ** n):
        got = zw.to_complex(st.vec[i], -st.k)
        assert abs(got - U[i, 0]) < 1e-10
        assert abs(sv.complex_state(text)[i] - U[i, 0]) < 1e-10


def test_statevector_closed_forms():
    # H on every qubit: every amplitude is 2^{-n/2}; GHZ: 1/sqrt2 on 0^n and 1^n
    n = 5
    text = "qubits 5\n" + "".join(f"h {q}\n" for q in range(n))
    for y in ["00000", "10110", "11111"]:
        assert sv.exact_amplitude(text, y) == ((1, 0, 0, 0), -5)
    ghz = "qubits 5\nh 0\n" + "".join(f"cx {q} {q + 1}\n" for q in range(n - 1))
    assert sv.exact_amplitude(ghz, "00000") == ((1, 0, 0, 0), -1)
    assert sv.exact_amplitude(ghz, "11111") == ((1, 0, 0, 0), -1)
    assert sv.exact_amplitude(ghz, "10000") == ((0, 0, 0, 0), 0)
    # H T H |0>: amplitude of 0 is (1 + w)/2
    assert sv.exact_amplitude("qubits 1\nh 0\nt 0\nh 0\n", "0") == zw.canonical((1, 1, 0, 0), -2)


def test_t_gate_identities():
    # T T = S, T^4 = Z, T^8 = I, T T^dag = I leave every amplitude unchanged
    rng = wl.SplitMix64(906, 0)
    c = wl.random_clifford_t(rng, 4, 40, 5)
    base = wl.circuit_text(c)
    g2 = []
    for g in c.gates:
        if g[0] == "s":
            g2 += [("t", g[1]), ("t", g[1])]
        else:
            g2.append(g)
    g2.insert(5, ("t", 0))
    g2.insert(6, ("tdg", 0))
    for _ in range(8):
        g2.insert(10, ("t", 2))
    text2 = wl.circuit_text(wl.circuits.Circuit(4, g2))
    for bits in itertools.product("01", repeat=4):
        y = "".join(bits)
        assert sv.exact_amplitude(base, y) == sv.exact_amplitude(text2, y)


@pytest.mark.parametrize("seed", range(3))
def test_born_rule_normalisation_exact(seed):
    rng = wl.SplitMix64(907, seed)
    n = 6
    c = wl.random_clifford_t(rng, n, 50, 8)
    text = wl.circuit_text(c)
    st = sv.exact_state(text)
    acc = zw.ZERO
    for z in st.vec:
        acc = zw.add(acc, zw.mul(z, zw.conj(z)))
    assert zw.canonical(acc, -2 * st.k) == ((1, 0, 0, 0), 0)
    for q in range(n):
        p0 = sv.exact_marginal(text, q, 0)
        p1 = sv.exact_marginal(text, q, 1)
        assert zw.add_scalar(*p0, *p1) == ((1, 0, 0, 0), 0)


# ----------------------------------------------------------------- marginals and weak sampling

def _bits(idx, k):
    return "".join("1" if idx >> i & 1 else "0" for i in range(k))


@pytest.mark.parametrize("seed", range(4))
def test_prefix_marginals_are_consistent(seed):
    # P over all prefixes of one length sums to 1, the one-qubit prefix is the single-qubit
    # marginal, the full-length prefix is |amp|^2, and P(B) = P(B0) + P(B1) (product rule)
    c, _ = wl.tiny_circuit(seed)
    text = wl.circuit_text(c)
    n = c.n_qubits
    for k in (1, 3, n):
        total = (zw.ZERO, 0)
        for idx in range(1 << k):
            total = zw.add_scalar(*total, *sv.exact_prefix_marginal(text, _bits(idx, k)))
        assert zw.canonical(*total) == (zw.ONE, 0)
    for v in (0, 1):
        assert sv.exact_prefix_marginal(text, str(v)) == sv.exact_marginal(text, 0, v)
    for idx in range(0, 1 << n, 7):
        y = _bits(idx, n)
        amp = sv.complex_amplitude(text, y)
        got = zw.to_complex(*sv.exact_prefix_marginal(text, y))
        assert abs(got - abs(amp) ** 2) < 1e-12
    for idx in range(1 << 3):
        b = _bits(idx, 3)
        whole = sv.exact_prefix_marginal(text, b)
        split = zw.add_scalar(*sv.exact_prefix_marginal(text, b + "0"), *sv.exact_prefix_marginal(text, b + "1"))
        assert zw.canonical(*split) == whole


def test_sign_of_a_plus_b_sqrt2_against_high_precision():
    import mpmath
    from oracle.sampling import sign_zsqrt2
    mpmath.mp.dps = 200
    r2 = mpmath.sqrt(2)
    rng = wl.SplitMix64(901, 0)
    cases = [(0, 0), (1, 0), (0, -1), (3, -2), (-3, 2), (7, -5), (-17, 12)]
    # Pell pairs: p^2 - 2 q^2 = +-1, so p - q sqrt2 is within 1/p of zero
    p, q = 1, 1
    for _ in range(60):
        cases += [(p, -q), (-p, q)]
        p, q = p + 2 * q, p + q
    def big(bits):  # uniform magnitude below 2^bits, random sign
        v = sum(rng.next_u64() << (64 * j) for j in range(3)) >> (192 - bits)
        return -v if rng.next_u64() & 1 else v
    for _ in range(300):
        bits = rng.randint(1, 190)
        cases.append((big(bits), big(bits)))
    for a, b in cases:
        want = mpmath.sign(mpmath.mpf(a) + mpmath.mpf(b) * r2)
        assert sign_zsqrt2(a, b) == int(want), (a, b)


def test_weak_samples_uniform_superposition():
    # H on every qubit: every conditional probability is 1/2, so bit k is 0 iff U < 2^52, and
    # every K-bit string has probability 2^-K
    from oracle.sampling import weak_samples
    n = 5
    text = "qubits 5\n" + "".join(f"h {q}\n" for q in range(n))
    u = wl.sampling_uniforms(0, 64, n)
    u[0, :] = (1 << 52) - 1
    u[1, :] = 1 << 52
    got, probs = weak_samples(text, u.tolist())
    for i, s in enumerate(got):
        assert s == "".join("0" if int(x) < (1 << 52) else "1" for x in u[i])
    assert all(pr == (zw.ONE, -2 * n) for pr in probs)


def test_weak_samples_basis_state():
    # a basis state is sampled with certainty, whatever the uniforms
    from oracle.sampling import weak_samples
    text = "qubits 4\nx 1\nh 2\nt 2\nh 2\nh 2\ntdg 2\nh 2\ncx 1 3\n"
    u = wl.sampling_uniforms(1, 50, 4)
    u[0, :] = (1 << 53) - 1
    u[1, :] = 0
    got, probs = weak_samples(text, u.tolist())
    assert set(got) == {"0101"} and all(p == (zw.ONE, 0) for p in probs)


def test_weak_samples_first_bit_is_the_marginal_threshold():
    # bit 0 is 0 exactly when U / 2^53 < P(y_0 = 0), computed here at high precision
    import mpmath
    from oracle.sampling import weak_samples
    mpmath.mp.dps = 100
    for seed in range(3):
        c, _ = wl.tiny_circuit(seed)
        text = wl.circuit_text(c)
        z, e = sv.exact_marginal(text, 0, 0)
        w = mpmath.exp(1j * mpmath.pi / 4)
        p0 = mpmath.re(sum(z[i] * w ** i for i in range(4)) * mpmath.sqrt(2) ** e)
        u = wl.sampling_uniforms(10 + seed, 200, 1)
        # two uniforms straddling the threshold as closely as 53 bits allow
        t = int(mpmath.floor(p0 * 2 ** 53))
        u[0, 0], u[1, 0] = t, min(t + 1, (1 << 53) - 1)
        got, _ = weak_samples(text, u.tolist(), 1)
        for i, s in enumerate(got):
            assert s == ("0" if mpmath.mpf(int(u[i, 0])) / 2 ** 53 < p0 else "1")


@pytest.mark.parametrize("seed", range(2))
def test_weak_samples_follow_the_exact_distribution(seed):
    # the chain rule samples each string with its Born probability: a chi-square test of 6000
    # samples against |amp|^2 (complex128 state vector); the threshold is the 0.999 quantile
    # for 63 degrees of freedom, and the inputs are fixed, so the outcome is deterministic
    from oracle.sampling import weak_samples
    c, _ = wl.tiny_circuit(seed)
    text = wl.circuit_text(c)
    n = c.n_qubits
    N = 6000
    got, probs = weak_samples(text, wl.sampling_uniforms(20 + seed, N, n).tolist())
    counts = np.zeros(1 << n)
    for s in got:
        counts[sv.index_of(s)] += 1
    p = np.abs(sv.complex_state(text)) ** 2
    keep = p * N >= 5
    chi2 = float(np.sum((counts[keep] - N * p[keep]) ** 2 / (N * p[keep])))
    assert counts[~keep].sum() <= max(20.0, 3 * N * p[~keep].sum())
    assert chi2 < 103.4, chi2
    # and each sample's reported probability is its own |amp|^2
    for s, pr in zip(got[:50], probs[:50]):
        assert abs(zw.to_complex(*pr) - p[sv.index_of(s)]) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_pattern_marginals(seed):
    # a pattern of fixed and free qubits: all free is 1, one fixed qubit is the single-qubit
    # marginal, a fixed prefix is the prefix marginal, all fixed is |amp|^2, and freeing a
    # qubit adds its two values
    c, _ = wl.tiny_circuit(seed)
    text = wl.circuit_text(c)
    n = c.n_qubits
    assert sv.exact_marginal_pattern(text, "*" * n) == (zw.ONE, 0)
    for q in range(n):
        for v in (0, 1):
            pat = "*" * q + str(v) + "*" * (n - q - 1)
            assert sv.exact_marginal_pattern(text, pat) == sv.exact_marginal(text, q, v)
    assert sv.exact_marginal_pattern(text, "101" + "*" * (n - 3)) == sv.exact_prefix_marginal(text, "101")
    y = "011010"[:n]
    amp = sv.complex_amplitude(text, y)
    assert abs(zw.to_complex(*sv.exact_marginal_pattern(text, y)) - abs(amp) ** 2) < 1e-12
    pat = "1*0*1*"[:n]
    both = zw.add_scalar(*sv.exact_marginal_pattern(text, pat.replace("*", "0", 1)),
                         *sv.exact_marginal_pattern(text, pat.replace("*", "1", 1)))
    assert zw.canonical(*both) == sv.exact_marginal_pattern(text, pat)
