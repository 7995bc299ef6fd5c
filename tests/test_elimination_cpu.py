"""Exact elimination of the vanishing conditions, host side (no GPU).

A node factor 1 + w^{a + b l(x)} with a or a + b = 4 (mod 8) is zero where its form takes one
value (the terms it kills, Section 5), so the nonzero terms lie on an affine subspace.  The
packer solves those conditions and sums over that subspace only; these tests check, with the
oracle, that the subspace it reports (sim_ir_affine_layout) holds every nonzero term: the
oracle's sum over its points equals the oracle's sum over all 2^p assignments.  They also pin
the oracle's point enumeration (--points) itself."""

import pytest

import paper_2403_06777_amd as zx
import workloads as wl
from workloads.programs import ProgramSpec


def gf2_rank(vectors):
    rows, rank = list(vectors), 0
    for bit in range(64):
        piv = next((i for i in range(rank, len(rows)) if rows[i] >> bit & 1), None)
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for i in range(len(rows)):
            if i != rank and rows[i] >> bit & 1:
                rows[i] ^= rows[rank]
        rank += 1
    return rank


def test_oracle_points_identity_and_affine_relabelling(o2):
    # --points with the unit columns is the plain enumeration; an invertible affine map of all
    # 2^p assignments permutes them and keeps the sum; half of a subspace plus the other half
    # (a range split) is the whole
    prog = wl.random_program(3, 9, n_nodes=8, n_pairs=1, n_lin=4, n_mono=10, scalar_range=2)
    text = prog.to_text()
    full = o2.evaluate(text)
    ident = o2.evaluate(text, points=(0, [1 << j for j in range(9)]))
    assert ident["raw"] == full["raw"]
    rows = wl.programs._random_invertible_rows(wl.SplitMix64(5, 1), 9)
    cols = [0] * 9
    for i in range(9):  # columns of the matrix whose rows are `rows`
        for j in range(9):
            if rows[i] >> j & 1:
                cols[j] |= 1 << i
    assert gf2_rank(cols) == 9
    moved = o2.evaluate(text, points=(0b101100101, cols))
    assert moved["raw"] == full["raw"]
    a = o2.evaluate(text, points=(0b11, cols[:5]), first=0, count=13)
    b = o2.evaluate(text, points=(0b11, cols[:5]), first=13, count=19)
    whole = o2.evaluate(text, points=(0b11, cols[:5]))
    assert tuple(x + y for x, y in zip(a["raw"], b["raw"])) == whole["raw"]
    # points outside the p parameters are refused
    with pytest.raises(RuntimeError):
        o2.evaluate(text, points=(1 << 9, [1]))


def _vanishing_programs():
    out = []
    for seed in range(12):
        p = 6 + seed % 9
        out.append(wl.kernel_sized_program(seed, p=p, n_factors=12 + 2 * p, n_monomials=4 * p).to_text())
    for seed in range(6):  # general (a, b): vanishing where a or a + b is 4
        out.append(wl.random_program(seed, 11, n_nodes=16, n_lin=5, n_mono=20, scalar_range=2).to_text())
    # planted: a node pair whose conditions contradict (no term survives)
    pr = ProgramSpec(7)
    f = pr.add_form(0, 0b1011001)
    g = pr.add_form(1, 0b0110100)
    h = pr.add_form(0, 0b1101101)  # f xor g xor 1
    pr.nodes += [(f, 4, 3), (g, 0, 4), (h, 4, 5), (pr.add_form(1, 0b11), 1, 2)]
    pr.mono = [(3, [0, 4]), (5, [1, 2, 6])]
    out.append(pr.to_text())
    return out


@pytest.mark.parametrize("k", range(19))
def test_subspace_holds_every_nonzero_term(o2, k):
    text = _vanishing_programs()[k]
    info = zx.sim_ir_info(text)
    kept = zx.sim_ir_info_flags(text, zx.binding.SIM_IR_KEEP_VANISHING)
    x0, cols = zx.sim_ir_affine_layout(text)
    p = info["n_params_given"]
    assert kept["n_params"] == p and kept["n_eliminated"] == 0
    assert info["n_params"] == p - info["n_eliminated"] == len(cols)
    assert gf2_rank(cols) == len(cols)
    assert x0 >> p == 0 and all(c >> p == 0 for c in cols)
    full = o2.evaluate(text)
    sub = o2.evaluate(text, points=(x0, cols))
    assert sub["raw"] == full["raw"]
    if info["n_eliminated"]:
        # the surviving fraction: 2^-rank of the vanishing conditions
        assert kept["nonzero_fraction"] == 2.0 ** -info["n_eliminated"] or info["is_zero"]


def test_contradicting_conditions_give_a_zero_program(o2):
    text = _vanishing_programs()[-1]
    assert o2.evaluate(text)["canonical"] == ((0, 0, 0, 0), 0)
    assert zx.sim_ir_info(text)["is_zero"] == 1


def test_kernel_sized_elimination_counts():
    # p = 32 with 11 (seed 0) and 12 (seed 1) independent vanishing conditions: 2^21 and 2^20
    # terms are summed; kept at run time they use the table of surviving steps instead
    for seed, rank in ((0, 11), (1, 12)):
        text = wl.kernel_sized_program(seed).to_text()
        info = zx.sim_ir_info(text)
        assert info["n_params_given"] == 32 and info["n_eliminated"] == rank
        assert info["n_params"] == 32 - rank
        assert info["n_form_monomials"] > 0 and 0 < info["n_mono_forms"] <= 32
        assert info["nonzero_fraction"] == 1.0 and info["vanish_table_bits"] == 0
        kept = zx.sim_ir_info_flags(text, zx.binding.SIM_IR_KEEP_VANISHING)
        assert kept["n_params"] == 32 and kept["vanish_table_bits"] == rank
        assert kept["nonzero_fraction"] == 2.0 ** -rank


def test_query_parameters_are_never_solved_for(o2):
    # a condition on the query (outer) parameters alone stays a run-time factor; one that also
    # has inner parameters is solved for an inner one
    pr = ProgramSpec(8)
    pr.nodes += [(pr.add_form(0, 0b11000000), 0, 4)]  # x6 xor x7: query parameters only
    pr.nodes += [(pr.add_form(1, 0b10001011), 4, 5)]
    pr.nodes += [(pr.add_form(0, 0b01110100), 3, 2)]
    pr.mono = [(1, [0, 6]), (6, [1, 3, 7])]
    text = pr.to_text().replace("p 8\n", "p 8\nouter 2\n")
    info = zx.sim_ir_info(text)
    assert info["n_eliminated"] == 0  # one condition has query parameters only: nothing solved
    pr.nodes = pr.nodes[1:]
    text = pr.to_text().replace("p 8\n", "p 8\nouter 2\n")
    info = zx.sim_ir_info(text)
    assert info["n_eliminated"] == 1 and info["n_outer"] == 2
    x0, cols = zx.sim_ir_affine_layout(text)
    # the query parameters keep the top two positions of the slice order
    assert (cols[-2] >> 6) & 3 == 1 and (cols[-1] >> 6) & 3 == 2
    assert all((c >> 6) & 3 == 0 for c in cols[:-2])
    assert o2.evaluate(text, points=(x0, cols))["raw"] == o2.evaluate(text)["raw"]
