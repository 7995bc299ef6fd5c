"""Repeated weak simulation by the chain rule: TEST INFRASTRUCTURE ONLY.

What it computes (the product rule of Section 2.2, used by the weak-simulation algorithm of
Appendix F): the bits of a sample are drawn in qubit order, and bit k is 0 exactly when
u_k < P(B || 0) / P(B), where B holds the bits drawn so far, P(prefix) is the probability that
the first len(prefix) qubits show that prefix, and u_k is uniform in [0, 1).  Here
u_k = U_k / 2^53 for a 53-bit integer U_k passed in, and the test U_k P(B) < 2^53 P(B || 0)
is decided exactly.

Probabilities come from the exact state vector: with amp_i = v_i sqrt2^{-h},
|amp_i|^2 = v_i conj(v_i) 2^{-h}, and v_i conj(v_i) is a real element a + b sqrt2 of Z[w]
(coefficients (a, b, 0, -b), since sqrt2 = w - w^3).  A marginal is a sum of those with the
same factor 2^{-h}, so every comparison is the sign of an integer combination a + b sqrt2,
decided with integers: the sign of a when b = 0 or a, b agree in sign, otherwise the sign of
a^2 - 2 b^2 taken with a's sign.
"""

from typing import Dict, List, Sequence, Tuple

from . import statevector as sv
from . import zomega as zw

U_BITS = 53


def real_coords(z: zw.ZW) -> Tuple[int, int]:
    """(a, b) with z = a + b sqrt2, for a real element z of Z[w]"""
    c0, c1, c2, c3 = z
    if c2 != 0 or c1 != -c3:
        raise ValueError("not a real element of Z[w]")
    return c0, c1


def sign_zsqrt2(a: int, b: int) -> int:
    """sign of a + b sqrt2 for integers a, b (sqrt2 is irrational, so 0 only when a = b = 0)"""
    if b == 0:
        return (a > 0) - (a < 0)
    if a == 0:
        return (b > 0) - (b < 0)
    if (a > 0) == (b > 0):
        return 1 if a > 0 else -1
    d = a * a - 2 * b * b  # never 0 for b != 0
    return (1 if d > 0 else -1) * (1 if a > 0 else -1)


class ExactDistribution:
    """The output distribution of a circuit: weights w_i = v_i conj(v_i) in Z[sqrt2] as (a, b)
    pairs, P(i) = (a + b sqrt2) 2^{-h}."""

    def __init__(self, text: str):
        st = sv.exact_state(text)
        self.n = st.n
        self.h = st.k
        self.w = [real_coords(zw.mul(z, zw.conj(z))) for z in st.vec]
        self._cache: Dict[Tuple[int, int], Tuple[int, int]] = {}

    def prefix_weight(self, k: int, prefix: int) -> Tuple[int, int]:
        """sum of the weights of every basis state whose first k bits are `prefix` (bit i of
        the integer = y_i)"""
        key = (k, prefix)
        if key not in self._cache:
            mask = (1 << k) - 1
            a = b = 0
            for i, (wa, wb) in enumerate(self.w):
                if i & mask == prefix:
                    a += wa
                    b += wb
            self._cache[key] = (a, b)
        return self._cache[key]

    def prefix_probability(self, k: int, prefix: int) -> Tuple[zw.ZW, int]:
        a, b = self.prefix_weight(k, prefix)
        return zw.canonical((a, b, 0, -b), -2 * self.h)


def weak_samples(text: str, uniforms: Sequence[Sequence[int]], k_max: int = -1) -> Tuple[List[str], List]:
    """One sample per row of `uniforms` (row i holds U_{i,0} .. U_{i,K-1}, each < 2^53), over
    the first K = k_max qubits (all when k_max < 0).  Returns the K-bit strings (character k =
    y_k) and each string's probability P(y_0 .. y_{K-1}) as a canonical (z, e)."""
    dist = ExactDistribution(text)
    K = dist.n if k_max < 0 else k_max
    out, probs = [], []
    for row in uniforms:
        if len(row) < K:
            raise ValueError("too few uniforms in a row")
        prefix = 0
        pa, pb = dist.prefix_weight(0, 0)  # the total weight 2^h
        for k in range(K):
            U = int(row[k])
            if not 0 <= U < (1 << U_BITS):
                raise ValueError("uniforms must be 53-bit integers")
            qa, qb = dist.prefix_weight(k + 1, prefix)  # bit k = 0
            # bit 0 iff U * P(B) < 2^53 * P(B || 0): the common 2^{-h} cancels
            if sign_zsqrt2((qa << U_BITS) - U * pa, (qb << U_BITS) - U * pb) > 0:
                pa, pb = qa, qb
            else:
                prefix |= 1 << k
                pa, pb = pa - qa, pb - qb
        out.append("".join("1" if prefix >> i & 1 else "0" for i in range(K)))
        probs.append(zw.canonical((pa, pb, 0, -pb), -2 * dist.h))
    return out, probs
