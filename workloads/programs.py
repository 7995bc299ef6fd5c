"""Random term programs in the ``zxir 1`` text format.

A term program denotes the parametric scalar

    S = sqrt2^e * c * sum_{x in {0,1}^p} w^{phi(x)} * prod_j F_j(x),      w = e^{i pi/4},

with F2-affine forms l_f(x) = const_f XOR parity(mask_f AND x), node factors
1 + w^{a + b*l(x)}, phase-pair factors 1 + w^{a+4 l1} + w^{b+4 l2} - w^{a+b+4(l1 XOR l2)}
(the subterm of the paper's Eq. 3 with Psi = a*pi/4 + pi*l1, Phi = b*pi/4 + pi*l2), and a
phase polynomial phi made of linear terms c*l_f(x) and variable monomials c*x_i*x_j*...

Text layout (counts first, sections in this order, ``#`` starts a comment)::

    zxir 1
    p <p>
    forms <F>        then F lines   f <const 0|1> <mask hex>      (bit i of mask = x_i)
    nodes <N>        then N lines   n <form> <a> <b>
    pairs <Q>        then Q lines   q <form1> <form2> <a> <b>
    lin <K>          then K lines   l <c> <form>
    mono <M>         then M lines   m <c> <d> <v_1> ... <v_d>
    scalar <c0> <c1> <c2> <c3> <e>     (c = c0 + c1 w + c2 w^2 + c3 w^3)
    end

Assignment index x = sum_i x_i 2^i.  Everything here is random drawing and text; the only
transformation is the relabelling x = A y XOR b of the variables (A invertible over F2),
which maps forms to forms and leaves the sum over all assignments unchanged.
"""

from dataclasses import dataclass, field
from typing import List, Tuple

from .rng import SplitMix64

STREAM_KERNEL_SIZED = 1
STREAM_RANDOM_PROGRAM = 11
STREAM_BLOCKS = 12


@dataclass
class ProgramSpec:
    p: int
    forms: List[Tuple[int, int]] = field(default_factory=list)       # (const, mask)
    nodes: List[Tuple[int, int, int]] = field(default_factory=list)  # (form, a, b)
    pairs: List[Tuple[int, int, int, int]] = field(default_factory=list)  # (f1, f2, a, b)
    lin: List[Tuple[int, int]] = field(default_factory=list)         # (c, form)
    mono: List[Tuple[int, List[int]]] = field(default_factory=list)  # (c, vars)
    scalar: Tuple[int, int, int, int] = (1, 0, 0, 0)
    sqrt2_exp: int = 0

    def add_form(self, const: int, mask: int) -> int:
        self.forms.append((const & 1, mask))
        return len(self.forms) - 1

    def to_text(self) -> str:
        out = ["zxir 1", f"p {self.p}", f"forms {len(self.forms)}"]
        out += [f"f {c} {m:x}" for c, m in self.forms]
        out.append(f"nodes {len(self.nodes)}")
        out += [f"n {f} {a} {b}" for f, a, b in self.nodes]
        out.append(f"pairs {len(self.pairs)}")
        out += [f"q {f1} {f2} {a} {b}" for f1, f2, a, b in self.pairs]
        out.append(f"lin {len(self.lin)}")
        out += [f"l {c} {f}" for c, f in self.lin]
        out.append(f"mono {len(self.mono)}")
        out += ["m {} {} {}".format(c, len(vs), " ".join(str(v) for v in vs)) for c, vs in self.mono]
        c = self.scalar
        out.append(f"scalar {c[0]} {c[1]} {c[2]} {c[3]} {self.sqrt2_exp}")
        out.append("end")
        return "\n".join(out) + "\n"


def _random_mask(rng: SplitMix64, p: int, density: float) -> int:
    m = 0
    for i in range(p):
        if rng.bernoulli(density):
            m |= 1 << i
    return m


def _random_monomials(rng: SplitMix64, p: int, count: int, max_deg: int = 3):
    """count monomials: degree U{1..max_deg} (capped at p), distinct variables,
    coefficient U{1..7}; repeated variable sets are merged mod 8 and dropped when 0."""
    merged = {}
    order = []
    for _ in range(count):
        d = min(rng.randint(1, max_deg), p)
        vs = tuple(sorted(rng.sample_distinct(p, d)))
        c = rng.randint(1, 7)
        if vs not in merged:
            merged[vs] = 0
            order.append(vs)
        merged[vs] = (merged[vs] + c) % 8
    return [(merged[vs], list(vs)) for vs in order if merged[vs] != 0]


def kernel_sized_program(seed: int, p: int = 32, n_factors: int = 64,
                         density: float = 0.3, n_monomials: int = 200) -> ProgramSpec:
    """Random parametric scalar of the kernel-sized workload: p Boolean parameters,
    n_factors node factors 1 + w^{k l(x)} with k uniform in {1..7} and l a random affine
    form (linear bits Bernoulli(density), constant bit Bernoulli(1/2)), and a phase
    polynomial of n_monomials random monomials of degree <= 3 with Z/8 coefficients."""
    rng = SplitMix64(STREAM_KERNEL_SIZED, seed)
    prog = ProgramSpec(p)
    for _ in range(n_factors):
        const = 1 if rng.bernoulli(0.5) else 0
        f = prog.add_form(const, _random_mask(rng, p, density))
        prog.nodes.append((f, 0, rng.randint(1, 7)))
    prog.mono = _random_monomials(rng, p, n_monomials)
    return prog


def random_program(seed: int, p: int, n_nodes: int = 8, n_pairs: int = 0, n_lin: int = 0,
                   n_mono: int = 0, density: float = 0.4, general_ab: bool = True,
                   max_deg: int = 3, scalar_range: int = 0, shared_forms: bool = False,
                   stream: int = STREAM_RANDOM_PROGRAM) -> ProgramSpec:
    """General random program for parity tests: node factors with (a, b) anywhere in Z8^2,
    phase-pair factors, linear phase terms over forms and variable monomials."""
    rng = SplitMix64(stream, seed * 1000003 + p)
    prog = ProgramSpec(p)
    n_forms = max(1, n_nodes + 2 * n_pairs + n_lin)
    if shared_forms:
        n_forms = max(1, n_forms // 2)
    for _ in range(n_forms):
        prog.add_form(1 if rng.bernoulli(0.5) else 0, _random_mask(rng, p, density) if p else 0)
    for _ in range(n_nodes):
        f = rng.randint(0, n_forms - 1)
        if general_ab:
            prog.nodes.append((f, rng.randint(0, 7), rng.randint(0, 7)))
        else:
            prog.nodes.append((f, 0, rng.randint(1, 7)))
    for _ in range(n_pairs):
        prog.pairs.append((rng.randint(0, n_forms - 1), rng.randint(0, n_forms - 1),
                           rng.randint(0, 7), rng.randint(0, 7)))
    for _ in range(n_lin):
        prog.lin.append((rng.randint(1, 7), rng.randint(0, n_forms - 1)))
    if p and n_mono:
        prog.mono = _random_monomials(rng, p, n_mono, max_deg)
    if scalar_range:
        prog.scalar = tuple(rng.randint(-scalar_range, scalar_range) for _ in range(4))
        prog.sqrt2_exp = rng.randint(-6, 6)
    return prog


def _random_invertible_rows(rng: SplitMix64, p: int) -> List[int]:
    """Rows of a random invertible p x p matrix over F2: the identity after 6p random
    row additions and swaps (each step is invertible, so the product is)."""
    rows = [1 << i for i in range(p)]
    for _ in range(6 * p):
        i = rng.randint(0, p - 1)
        j = rng.randint(0, p - 1)
        if i == j:
            continue
        if rng.bernoulli(0.8):
            rows[i] ^= rows[j]
        else:
            rows[i], rows[j] = rows[j], rows[i]
    return rows


def _parity(v: int) -> int:
    return bin(v).count("1") & 1


def block_separable_program(seed: int, p: int, block_size: int = 4, factors_per_block: int = 2,
                            lin_per_block: int = 1, mono_per_block: int = 0,
                            pairs_per_block: int = 0, scramble: bool = True, no_vanishing: bool = False):
    """A program whose variables split into independent blocks of <= block_size, so its
    sum is the product of the block sums; then relabelled by x = A y XOR b.

    Returns (program, blocks): each block is a small ProgramSpec over its own variables.
    With ``scramble`` the relabelling is a random invertible affine map (allowed only when
    there are no variable monomials, since a monomial in x is not a monomial in y); with
    monomials the relabelling is a random permutation of the variables plus a shift b.
    no_vanishing redraws node factors until neither of their two values is 1 + w^4 = 0 (so every
    block sum is large: the int128 stress cases)."""
    if mono_per_block and scramble:
        raise ValueError("variable monomials only survive a permutation relabelling")
    rng = SplitMix64(STREAM_BLOCKS, seed * 7919 + p)
    blocks = []
    full = ProgramSpec(p)
    start = 0
    while start < p:
        size = min(block_size, p - start)
        blk = ProgramSpec(size)
        for _ in range(factors_per_block):
            const = 1 if rng.bernoulli(0.5) else 0
            mask = _random_mask(rng, size, 0.6) or 1
            f = blk.add_form(const, mask)
            a, b = rng.randint(0, 7), rng.randint(1, 7)
            while no_vanishing and (a == 4 or (a + b) % 8 == 4):
                a, b = rng.randint(0, 7), rng.randint(1, 7)
            blk.nodes.append((f, a, b))
        for _ in range(pairs_per_block):
            f1 = blk.add_form(rng.randint(0, 1), _random_mask(rng, size, 0.6) or 1)
            f2 = blk.add_form(rng.randint(0, 1), _random_mask(rng, size, 0.6) or 1)
            blk.pairs.append((f1, f2, rng.randint(0, 7), rng.randint(0, 7)))
        for _ in range(lin_per_block):
            f = blk.add_form(rng.randint(0, 1), _random_mask(rng, size, 0.6) or 1)
            blk.lin.append((rng.randint(1, 7), f))
        if mono_per_block:
            blk.mono = _random_monomials(rng, size, mono_per_block)
        blocks.append((start, blk))
        start += size

    # embed the blocks side by side in x
    for off, blk in blocks:
        base = len(full.forms)
        for c, m in blk.forms:
            full.forms.append((c, m << off))
        full.nodes += [(base + f, a, b) for f, a, b in blk.nodes]
        full.pairs += [(base + f1, base + f2, a, b) for f1, f2, a, b in blk.pairs]
        full.lin += [(c, base + f) for c, f in blk.lin]
        full.mono += [(c, [v + off for v in vs]) for c, vs in blk.mono]

    b = _random_mask(rng, p, 0.5)
    if scramble:
        rows = _random_invertible_rows(rng, p)  # x_i = parity(rows[i] & y) XOR b_i
        new_forms = []
        for c, m in full.forms:
            mm = 0
            for i in range(p):
                if m >> i & 1:
                    mm ^= rows[i]
            new_forms.append((c ^ _parity(m & b), mm))
        full.forms = new_forms
    else:
        perm = list(range(p))
        for i in range(p - 1, 0, -1):  # Fisher-Yates; x_i = y_perm[i] XOR b_i
            j = rng.randint(0, i)
            perm[i], perm[j] = perm[j], perm[i]
        # a monomial prod x_i stays a monomial only if none of its variables is flipped
        used = 0
        for _, vs in full.mono:
            for v in vs:
                used |= 1 << v
        b &= ~used
        new_forms = []
        for c, m in full.forms:
            mm = 0
            for i in range(p):
                if m >> i & 1:
                    mm |= 1 << perm[i]
            new_forms.append((c ^ _parity(m & b), mm))
        full.forms = new_forms
        full.mono = [(c, sorted(perm[v] for v in vs)) for c, vs in full.mono]
    return full, [blk for _, blk in blocks]


def appendix_d_terms() -> List[ProgramSpec]:
    """The worked example of the paper's Appendix D (coalescing): 4 parameters and two
    terms of phase-pair subterms, each row (flag, 4 alpha/pi, P^psi bits, 4 beta/pi,
    P^phi bits).  Row 3 is a dummy (flag 0) and is left out.  Parameter p_k is x_{k-1}.
    Returns one program per term; the example's scalar is their sum with C_1 = C_2 = 1."""
    rows = [
        # flag, a, psi bits p1..p4, b, phi bits p1..p4
        (1, 2, (1, 1, 0, 0), 7, (1, 1, 1, 0)),
        (1, 4, (0, 1, 1, 1), 3, (0, 1, 0, 1)),
        (0, 0, (0, 0, 0, 0), 0, (0, 0, 0, 0)),
        (1, 6, (1, 0, 0, 0), 3, (1, 1, 1, 1)),
        (1, 5, (1, 1, 1, 1), 1, (1, 0, 1, 0)),
        (1, 2, (0, 0, 0, 1), 4, (1, 1, 0, 0)),
    ]
    terms = []
    for group in (rows[0:3], rows[3:6]):
        prog = ProgramSpec(4)
        for flag, a, psi, b, phi in group:
            if not flag:
                continue
            m1 = sum(bit << k for k, bit in enumerate(psi))
            m2 = sum(bit << k for k, bit in enumerate(phi))
            f1 = prog.add_form(0, m1)
            f2 = prog.add_form(0, m2)
            prog.pairs.append((f1, f2, a, b))
        terms.append(prog)
    return terms


def block_bound_program(n_nodes: int, p: int = 14) -> ProgramSpec:
    """n_nodes node factors 1 + w^l on the top parameter, and 12 linear terms on forms of the
    top parameter and parameters p-6 .. p-3 (parameters below p-6 enter no form).  Where the
    top parameter is 0, every term is 2^n_nodes times a phase that depends only on parameters
    p-6 .. p-3, so any 64 consecutive assignments of the low parameters sum to 2^(n_nodes+6)
    times that phase."""
    prog = ProgramSpec(p)
    f = prog.add_form(0, 1 << (p - 1))
    for _ in range(n_nodes):
        prog.nodes.append((f, 0, 1))
    for m in range(1, 13):
        prog.lin.append((2 * (m % 4) + 1, prog.add_form(0, (1 << (p - 1)) | (m << (p - 6)))))
    return prog


def weight4_phase_program(seed: int, p: int, n_nodes: int, case: str) -> ProgramSpec:
    """Programs whose linear phase terms carry weight-4 parts (coefficients 4..7) in the ways
    they can combine: `random` (many terms with coefficients 1..7, half of them on forms
    already there, the node factors' included), `node` (the parts' forms add up to a node
    factor's form), `opposite` (they add up to another linear term's form with the other
    constant), `constant` (they add up to the constant 1)."""
    rng = SplitMix64(STREAM_RANDOM_PROGRAM, 7_000_003 + seed * 1009 + p * 31 + n_nodes)
    prog = ProgramSpec(p)

    def mask():
        m = _random_mask(rng, p, 0.4)
        return m if m else 1 << rng.randint(0, p - 1)

    for _ in range(n_nodes):
        f = prog.add_form(rng.randint(0, 1), mask())
        prog.nodes.append((f, rng.randint(0, 7), rng.randint(1, 7)))
    if case == "random":
        for _ in range(3 * p):
            if prog.forms and rng.bernoulli(0.5):
                f = rng.randint(0, len(prog.forms) - 1)
            else:
                f = prog.add_form(rng.randint(0, 1), mask())
            prog.lin.append((rng.randint(1, 7), f))
    else:
        a = prog.add_form(rng.randint(0, 1), mask())
        b = prog.add_form(rng.randint(0, 1), mask())
        ca, ma = prog.forms[a]
        cb, mb = prog.forms[b]
        prog.lin += [(4, a), (5, b)]
        if case == "node":
            c0, m0 = prog.forms[0]
            c = prog.add_form(c0 ^ ca ^ cb ^ rng.randint(0, 1), m0 ^ ma ^ mb)
            prog.lin.append((4, c))
        elif case == "opposite":
            d = prog.add_form(ca ^ cb ^ 1, ma ^ mb)
            prog.lin.append((rng.randint(1, 3), d))
        elif case == "constant":
            prog.lin.append((4, prog.add_form(cb ^ 1, mb)))
            prog.lin.append((4, prog.add_form(ca, ma)))
        else:
            raise ValueError(case)
        for _ in range(p // 2):  # terms without a weight-4 part
            prog.lin.append((rng.randint(1, 3), prog.add_form(rng.randint(0, 1), mask())))
    return prog
