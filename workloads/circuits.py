"""Random Clifford+T circuits: the benchmark family of the paper's Section 4.

The paper strongly simulates "randomly generated Clifford+T circuits of various T-counts"
without fixing a recipe.  The recipe used here:

* ``n_clifford`` gates drawn i.i.d. and uniformly from {H, S, CNOT}; an H or S acts on a
  uniform qubit, a CNOT on an ordered pair of distinct uniform qubits;
* ``n_t`` T gates, each inserted at a uniform position of the growing gate list and on a
  uniform qubit, so the total gate count is ``n_clifford + n_t``.

Circuit text format, one gate per line (``#`` starts a comment)::

    qubits <n>
    h <q> | s <q> | sdg <q> | t <q> | tdg <q> | z <q> | x <q>
    cx <control> <target> | cz <a> <b>

Qubit ``i`` of an output bit string ``y`` is character ``i`` of the string.
"""

from dataclasses import dataclass, field
from typing import List, Tuple

from .rng import SplitMix64

# generator stream per workload family, so the families never share draws
STREAM_TINY = 0
STREAM_CIRCUIT_SCALE = 2
STREAM_BATCH = 3
STREAM_SERVING = 4
STREAM_SAMPLING = 5


@dataclass
class Circuit:
    n_qubits: int
    gates: List[Tuple] = field(default_factory=list)

    @property
    def t_count(self) -> int:
        return sum(1 for g in self.gates if g[0] in ("t", "tdg"))


def random_clifford_t(rng: SplitMix64, n_qubits: int, n_clifford: int, n_t: int) -> Circuit:
    gates: List[Tuple] = []
    for _ in range(n_clifford):
        kind = rng.randint(0, 2)
        if kind == 0:
            gates.append(("h", rng.randint(0, n_qubits - 1)))
        elif kind == 1:
            gates.append(("s", rng.randint(0, n_qubits - 1)))
        else:
            if n_qubits < 2:
                gates.append(("h", 0))
                continue
            c, t = rng.sample_distinct(n_qubits, 2)
            gates.append(("cx", c, t))
    for _ in range(n_t):
        pos = rng.randint(0, len(gates))
        gates.insert(pos, ("t", rng.randint(0, n_qubits - 1)))
    return Circuit(n_qubits, gates)


def circuit_text(c: Circuit) -> str:
    lines = [f"qubits {c.n_qubits}"]
    for g in c.gates:
        lines.append(" ".join(str(v) for v in g))
    return "\n".join(lines) + "\n"


def random_bits(rng: SplitMix64, n: int) -> str:
    return "".join("1" if rng.bernoulli(0.5) else "0" for _ in range(n))


def tiny_circuit(seed: int) -> Tuple[Circuit, str]:
    """6 qubits, 60 Clifford gates from {H,S,CNOT}, 8 T gates; query <0^6|C|0^6>."""
    rng = SplitMix64(STREAM_TINY, seed)
    return random_clifford_t(rng, 6, 60, 8), "0" * 6


def circuit_scale(seed: int) -> Tuple[Circuit, str]:
    """24 qubits, 600 Clifford gates, 40 T gates; amplitude of a random output string."""
    rng = SplitMix64(STREAM_CIRCUIT_SCALE, seed)
    c = random_clifford_t(rng, 24, 600, 40)
    return c, random_bits(rng, 24)


def batch_queries(n: int = 512, base_seed: int = 0):
    """Amplitude queries of uneven size: qubits U{10..40}, Clifford gates U{200..1000},
    T count U{10..50}, random output string; seed = query index."""
    out = []
    for i in range(n):
        rng = SplitMix64(STREAM_BATCH, base_seed + i)
        nq = rng.randint(10, 40)
        ng = rng.randint(200, 1000)
        nt = rng.randint(10, 50)
        c = random_clifford_t(rng, nq, ng, nt)
        out.append((c, random_bits(rng, nq)))
    return out


def serving_pool(n_circuits: int = 64, base_seed: int = 0):
    """Circuit pool for the serving stream: qubits U{20..50}, T count U{20..80},
    Clifford gates U{200..1000}."""
    pool = []
    for i in range(n_circuits):
        rng = SplitMix64(STREAM_SERVING, base_seed + i)
        nq = rng.randint(20, 50)
        nt = rng.randint(20, 80)
        ng = rng.randint(200, 1000)
        pool.append(random_clifford_t(rng, nq, ng, nt))
    return pool


def sampling_circuit(seed: int, n_qubits: int = 20, n_clifford: int = 400, n_t: int = 32) -> Circuit:
    """Circuit for repeated weak simulation (every qubit measured, one bit at a time)."""
    return random_clifford_t(SplitMix64(STREAM_SAMPLING, seed), n_qubits, n_clifford, n_t)


def sampling_uniforms(seed: int, n_samples: int, k: int):
    """n_samples x k table of 53-bit integers U (the uniform u = U / 2^53 in [0, 1)), row i
    for sample i; uint64 numpy array, equal to drawing SplitMix64(STREAM_SAMPLING + 100, seed)
    row by row and taking the top 53 bits of each output."""
    from .rng import splitmix64_array
    return (splitmix64_array(STREAM_SAMPLING + 100, seed, n_samples * k) >> 11).reshape(n_samples, k)
