"""Dense state-vector simulation of Clifford+T circuits: TEST INFRASTRUCTURE ONLY.

This is the plain definition that the parametric method reaches by other means
(Section 2.2: an amplitude is the scalar of the circuit closed with the input state and
the effect of an outcome; a probability is |amplitude|^2 by the Born rule; a single-qubit
marginal is <0^n| C^dag (|a><a|_q (x) I) C |0^n>, the "doubling" form of Fig. 3).

Two simulators, sharing nothing with the GPU library:

* ``ExactState`` holds every amplitude as an element of Z[w] with one common factor
  sqrt2^{-k} (k = number of H gates so far): H maps (u, v) to (u + v, u - v) and raises k,
  S and T rotate the |1> component by w^2 and w, CNOT permutes.  No rounding anywhere;
  meant for n <= 14.
* ``complex_state`` is the same circuit in complex128 with numpy, for tolerance checks of
  larger circuits (n <= 26).

Circuit text: ``qubits n`` then one gate per line among h s sdg t tdg z x (one qubit) and
cx cz (two qubits).  Basis index of a bit string y is sum_i y_i 2^i.
"""

from typing import List, Tuple

import numpy as np

from . import zomega as zw

ONE_QUBIT = {"h", "s", "sdg", "t", "tdg", "z", "x"}
TWO_QUBIT = {"cx", "cz"}
# phase exponent (in units of w = e^{i pi/4}) applied to |1> by each diagonal gate
DIAG_PHASE = {"s": 2, "sdg": 6, "t": 1, "tdg": 7, "z": 4}


def parse_circuit(text: str) -> Tuple[int, List[Tuple]]:
    n = None
    gates = []
    for lineno, raw in enumerate(text.splitlines(), 1):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "qubits":
            n = int(tok[1])
            continue
        if n is None:
            raise ValueError(f"line {lineno}: gate before 'qubits'")
        name = tok[0].lower()
        args = [int(v) for v in tok[1:]]
        if name in ONE_QUBIT and len(args) == 1 or name in TWO_QUBIT and len(args) == 2:
            if any(a < 0 or a >= n for a in args) or (len(args) == 2 and args[0] == args[1]):
                raise ValueError(f"line {lineno}: bad qubit")
            gates.append((name, *args))
        else:
            raise ValueError(f"line {lineno}: unknown gate '{line}'")
    if n is None:
        raise ValueError("missing 'qubits'")
    return n, gates


def inverse_gates(gates: List[Tuple]) -> List[Tuple]:
    """C^dagger as a gate list: reversed order, each gate replaced by its adjoint"""
    adj = {"s": "sdg", "sdg": "s", "t": "tdg", "tdg": "t"}
    return [(adj.get(g[0], g[0]),) + tuple(g[1:]) for g in reversed(gates)]


class ExactState:
    """State sum_i amp[i] |i> with amp[i] = vec[i] * sqrt2^{-k}, vec[i] in Z[w]."""

    def __init__(self, n: int):
        if n > 16:
            raise ValueError("exact state vector is meant for small n")
        self.n = n
        self.vec = [zw.ZERO] * (1 << n)
        self.vec[0] = zw.ONE
        self.k = 0

    def apply(self, g: Tuple):
        name = g[0]
        vec = self.vec
        if name == "h":
            bit = 1 << g[1]
            for i in range(len(vec)):
                if not i & bit:
                    u, v = vec[i], vec[i | bit]
                    vec[i], vec[i | bit] = zw.add(u, v), zw.sub(u, v)
            self.k += 1
        elif name in DIAG_PHASE:
            bit = 1 << g[1]
            ph = zw.omega_pow(DIAG_PHASE[name])
            for i in range(len(vec)):
                if i & bit:
                    vec[i] = zw.mul(vec[i], ph)
        elif name == "x":
            bit = 1 << g[1]
            for i in range(len(vec)):
                if not i & bit:
                    vec[i], vec[i | bit] = vec[i | bit], vec[i]
        elif name == "cx":
            cb, tb = 1 << g[1], 1 << g[2]
            for i in range(len(vec)):
                if i & cb and not i & tb:
                    vec[i], vec[i | tb] = vec[i | tb], vec[i]
        elif name == "cz":
            ab, bb = 1 << g[1], 1 << g[2]
            for i in range(len(vec)):
                if i & ab and i & bb:
                    vec[i] = zw.neg(vec[i])
        else:
            raise ValueError(name)

    def run(self, gates):
        for g in gates:
            self.apply(g)
        return self


def index_of(bits: str) -> int:
    return sum(1 << i for i, ch in enumerate(bits) if ch == "1")


def exact_amplitude(text: str, out_bits: str) -> Tuple[zw.ZW, int]:
    """<y|C|0^n> as a canonical (z, e): value z * sqrt2^e"""
    n, gates = parse_circuit(text)
    if len(out_bits) != n:
        raise ValueError("output string length != qubit count")
    st = ExactState(n).run(gates)
    return zw.canonical(st.vec[index_of(out_bits)], -st.k)


def exact_marginal(text: str, qubit: int, value: int) -> Tuple[zw.ZW, int]:
    """P(qubit = value) = sum over basis states with that bit of |amp|^2, exactly"""
    n, gates = parse_circuit(text)
    st = ExactState(n).run(gates)
    acc = zw.ZERO
    for i, z in enumerate(st.vec):
        if (i >> qubit & 1) == value:
            acc = zw.add(acc, zw.mul(z, zw.conj(z)))
    return zw.canonical(acc, -2 * st.k)


def exact_prefix_marginal(text: str, prefix: str) -> Tuple[zw.ZW, int]:
    """P(y_0 .. y_{k-1} = prefix), k = len(prefix): the sum of |amp|^2 over every basis state
    whose first k bits are the prefix (the summing form of a marginal, Fig. 3 left), exactly"""
    n, gates = parse_circuit(text)
    st = ExactState(n).run(gates)
    k = len(prefix)
    want = index_of(prefix)
    acc = zw.ZERO
    for i, z in enumerate(st.vec):
        if i & ((1 << k) - 1) == want:
            acc = zw.add(acc, zw.mul(z, zw.conj(z)))
    return zw.canonical(acc, -2 * st.k)


def exact_marginal_pattern(text: str, pattern: str) -> Tuple[zw.ZW, int]:
    """P(y_i = pattern[i] wherever pattern[i] is '0' or '1'): the sum of |amp|^2 over every
    basis state that agrees with the pattern, a '*' leaving its qubit free (Fig. 3 left)"""
    n, gates = parse_circuit(text)
    if len(pattern) != n:
        raise ValueError("pattern length != qubit count")
    st = ExactState(n).run(gates)
    acc = zw.ZERO
    for i, z in enumerate(st.vec):
        if all(ch == "*" or (i >> q & 1) == int(ch) for q, ch in enumerate(pattern)):
            acc = zw.add(acc, zw.mul(z, zw.conj(z)))
    return zw.canonical(acc, -2 * st.k)


def exact_state(text: str) -> ExactState:
    n, gates = parse_circuit(text)
    return ExactState(n).run(gates)


def complex_state(text: str) -> np.ndarray:
    """complex128 state vector; axis n-1-q of the (2,)*n tensor is qubit q, so the flat
    index of a basis state is sum_q y_q 2^q.  Gates update views of the tensor in place."""
    import torch  # plain CPU tensor ops (multithreaded); no GPU involved

    n, gates = parse_circuit(text)
    if n > 26:
        raise ValueError("too many qubits for a dense complex state")
    psi = torch.zeros((2,) * n, dtype=torch.complex128)
    psi[(0,) * n] = 1.0
    s = 1 / np.sqrt(2)
    phases = {k: complex(np.exp(1j * np.pi * v / 4)) for k, v in DIAG_PHASE.items()}

    def sl(**fixed):  # index tuple fixing some qubits to 0/1
        idx = [slice(None)] * n
        for q, v in fixed.items():
            idx[n - 1 - int(q[1:])] = v
        return tuple(idx)

    for g in gates:
        name = g[0]
        if name == "h":
            x0 = psi[sl(**{f"q{g[1]}": 0})]
            x1 = psi[sl(**{f"q{g[1]}": 1})]
            tmp = x0.clone()
            x0 += x1
            x0 *= s
            x1 -= tmp
            x1 *= -s
        elif name in phases:
            psi[sl(**{f"q{g[1]}": 1})] *= phases[name]
        elif name == "x":
            x0 = psi[sl(**{f"q{g[1]}": 0})]
            x1 = psi[sl(**{f"q{g[1]}": 1})]
            tmp = x0.clone()
            x0.copy_(x1)
            x1.copy_(tmp)
        elif name == "cx":
            a = psi[sl(**{f"q{g[1]}": 1, f"q{g[2]}": 0})]
            b = psi[sl(**{f"q{g[1]}": 1, f"q{g[2]}": 1})]
            tmp = a.clone()
            a.copy_(b)
            b.copy_(tmp)
        elif name == "cz":
            psi[sl(**{f"q{g[1]}": 1, f"q{g[2]}": 1})] *= -1
    return psi.reshape(-1).numpy()


def complex_amplitude(text: str, out_bits: str) -> complex:
    psi = complex_state(text)
    return complex(psi[index_of(out_bits)])
