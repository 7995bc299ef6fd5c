"""SplitMix64, the counter-based generator every seeded input is drawn from.

Definition (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014): the state advances by the golden-ratio increment 0x9E3779B97F4A7C15 and
each output is the state passed through the variant-13 finaliser of MurmurHash3.
"""

MASK64 = (1 << 64) - 1


class SplitMix64:
    """Deterministic 64-bit generator keyed by (stream, seed)."""

    def __init__(self, stream: int, seed: int):
        # key the state by both integers, then mix once so nearby keys diverge
        self.state = ((stream & 0xFFFFFFFF) << 32 | (seed & 0xFFFFFFFF)) & MASK64
        self.next_u64()

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive), by rejection so it is unbiased."""
        span = hi - lo + 1
        if span <= 0:
            raise ValueError("empty range")
        limit = (1 << 64) - ((1 << 64) % span)
        while True:
            r = self.next_u64()
            if r < limit:
                return lo + r % span

    def bernoulli(self, q: float) -> bool:
        return self.next_u64() < int(q * (1 << 64))

    def uniform(self) -> float:
        """Uniform float in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def choice(self, seq):
        return seq[self.randint(0, len(seq) - 1)]

    def sample_distinct(self, n: int, k: int):
        """k distinct integers from range(n), in draw order."""
        out = []
        seen = set()
        while len(out) < k:
            v = self.randint(0, n - 1)
            if v not in seen:
                seen.add(v)
                out.append(v)
        return out


def splitmix64_array(stream: int, seed: int, count: int):
    """The first `count` outputs of SplitMix64(stream, seed) as a uint64 numpy array (the
    generator is counter-based: output j comes from state key + (j + 2) * increment, the +1
    being the mixing draw of the constructor)."""
    import numpy as np
    key = np.uint64(((stream & 0xFFFFFFFF) << 32 | (seed & 0xFFFFFFFF)) & MASK64)
    with np.errstate(over="ignore"):
        z = key + np.uint64(0x9E3779B97F4A7C15) * np.arange(2, count + 2, dtype=np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))
