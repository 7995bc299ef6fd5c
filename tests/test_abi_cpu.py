"""The C-ABI library loads, exports every declared symbol, and its host-only paths
(IR parsing, packing, error reporting) behave as documented.  No GPU needed."""

import ctypes

import pytest

import paper_2403_06777_amd as zx
import workloads as wl
from paper_2403_06777_amd import binding
from tests.helpers import header_functions


def test_library_exports_every_declared_function():
    lib = binding.lib()
    declared = header_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    bound = {name for name, _, _ in binding.SIGNATURES}
    assert set(declared) == bound


def test_binding_exposes_c_names():
    for name in header_functions():
        assert hasattr(zx, name) or name in ("sim_last_error",), name


def wide_vanishing_program(seed, p=24, n_vanish=36, basis=6):
    # more than 32 factors that can vanish (their bits of L span two words), on forms from a
    # small subspace so that a fraction 2^-basis of the terms survives
    from workloads.programs import ProgramSpec
    rng = wl.SplitMix64(80, seed)
    base = [rng.randint(1, (1 << p) - 1) for _ in range(basis)]
    star = rng.randint(0, (1 << p) - 1)  # every vanishing form is 0 (factor 2) here
    prog = ProgramSpec(p)
    for _ in range(n_vanish):
        m = 0
        while m == 0:
            m = 0
            for b in base:
                if rng.bernoulli(0.5):
                    m ^= b
        prog.nodes.append((prog.add_form(bin(m & star).count("1") & 1, m), 0, 4))
    for _ in range(12):
        prog.nodes.append((prog.add_form(rng.randint(0, 1), rng.randint(1, (1 << p) - 1)), rng.randint(0, 7), rng.randint(1, 7)))
    for _ in range(20):
        prog.mono.append((rng.randint(1, 7), sorted(rng.sample_distinct(p, rng.randint(1, 3)))))
    return prog


def test_vanishing_step_table_is_reported():
    # kept at run time, vanishing factors whose bits all lie in word 0 use the table of
    # surviving steps (the kernel-sized programs: 11 and 12 of them); more than 32 use the
    # reduced-basis test; programs without vanishing factors report 0
    keep = zx.binding.SIM_IR_KEEP_VANISHING
    assert zx.sim_ir_info_flags(wl.kernel_sized_program(0).to_text(), keep)["vanish_table_bits"] == 11
    assert zx.sim_ir_info_flags(wl.kernel_sized_program(1).to_text(), keep)["vanish_table_bits"] == 12
    assert zx.sim_ir_info_flags(wide_vanishing_program(0).to_text(), keep)["vanish_table_bits"] == 0
    assert zx.sim_ir_info(wl.random_program(0, 10, n_nodes=0, n_lin=8).to_text())["vanish_table_bits"] == 0


def test_ir_info_kernel_sized():
    prog = wl.kernel_sized_program(0)
    info = zx.sim_ir_info_flags(prog.to_text(), zx.binding.SIM_IR_KEEP_VANISHING)
    assert info["n_params"] == 32
    assert info["n_factors"] == 64
    assert info["n_monomials"] == len(prog.mono)
    assert info["n_slices"] << info["walk_bits"] == 1 << 32
    info = zx.sim_ir_info(prog.to_text())  # the 11 vanishing factors solved for
    assert info["n_params"] == 21 and info["n_factors"] == 53
    assert info["n_slices"] << info["walk_bits"] == 1 << 21
    # 147 form monomials, all of them in LDS: two-wave teams; 53 factors allow no 32-bit sums
    assert info["n_form_monomials"] == 147 and info["team_waves"] == 2
    assert info["block_sum32"] == 0


@pytest.mark.parametrize("text,frag", [
    ("zxir 2\n", "range"),
    ("zxir 1\np 3\nforms 1\nf 0 ff\n", "parameter >= p"),
    ("zxir 1\np 3\nforms 1\nf 0 1\nnodes 1\nn 4 0 1\n", "out of range"),
    ("zxir 1\np 3\nforms 0\nnodes 0\npairs 0\nlin 0\nmono 0\nscalar 1 0 0 0 0\n", "end of program"),
    ("zxir 1\np 3\nforms 0\nnodes 0\npairs 0\nlin 0\nmono 0\nscalar 1 0 0 0 0\nend\nextra\n", "after 'end'"),
    ("zxir 1\np 70\n", "out of range"),
    ("zxir 1\np 2\nforms 0\nnodes 0\npairs 0\nlin 0\nmono 1\nm 1 1 5\nscalar 1 0 0 0 0\nend\n", "out of range"),
])
def test_ir_errors_are_reported(text, frag):
    with pytest.raises(zx.SimError) as ei:
        zx.sim_ir_info(text)
    assert ei.value.code == binding.SIM_EINVAL
    assert frag in str(ei.value)


def test_error_names_line():
    text = "zxir 1\np 3\nforms 1\nf 0 1\nnodes 1\nn 0 x 1\n"
    with pytest.raises(zx.SimError) as ei:
        zx.sim_ir_info(text)
    assert "line 6" in str(ei.value)


def test_static_bound_refuses_overflow():
    # 80 node factors over 60 parameters: the bound 2^(factors + p) exceeds int128 with the 12
    # vanishing factors kept; solved for, 68 factors and parameters go and the program fits
    prog = wl.random_program(0, 60, n_nodes=80, general_ab=False)
    with pytest.raises(zx.SimError) as ei:
        zx.sim_ir_info_flags(prog.to_text(), binding.SIM_IR_KEEP_VANISHING)
    assert ei.value.code == binding.SIM_ERANGE
    info = zx.sim_ir_info(prog.to_text())
    assert info["n_eliminated"] == 12 and info["n_params"] + info["n_factors"] <= 125
    # no factor can vanish: 80 factors + 60 parameters > 125 is refused either way
    from workloads.programs import ProgramSpec
    rng = wl.SplitMix64(84, 0)
    prog = ProgramSpec(60)
    for _ in range(80):
        prog.nodes.append((prog.add_form(rng.randint(0, 1), rng.randint(1, (1 << 60) - 1)), 0,
                           rng.choice([1, 2, 3, 5, 6, 7])))
    with pytest.raises(zx.SimError) as ei:
        zx.sim_ir_info(prog.to_text())
    assert ei.value.code == binding.SIM_ERANGE


def test_constant_factors_fold_and_zero_program():
    prog = wl.ProgramSpec(3)
    f = prog.add_form(1, 0)   # constant 1
    prog.nodes = [(f, 0, 4)]  # 1 + w^4 = 0
    info = zx.sim_ir_info(prog.to_text())
    assert info["is_zero"] == 1
    prog.nodes = [(f, 0, 2)]  # 1 + w^2, folded into the constant
    info = zx.sim_ir_info(prog.to_text())
    assert info["is_zero"] == 0 and info["n_factors"] == 0


def test_pairs_add_walk_parameters():
    t = wl.appendix_d_terms()[1]
    info = zx.sim_ir_info(t.to_text())
    assert info["n_params"] == 4
    assert info["n_eval_params"] == 4 + len(t.pairs)


def test_many_forms_pick_wider_vectors():
    prog = wl.random_program(1, 20, n_nodes=40, n_lin=300)
    info = zx.sim_ir_info(prog.to_text())
    assert info["n_forms"] > 128


def test_raw_add_is_exact_and_checks_overflow():
    a = (2 ** 100, -5, 3, -(2 ** 90))
    b = (2 ** 100, 7, -3, 2 ** 90 + 1)
    assert zx.sim_raw_add(a, b) == (2 ** 101, 2, 0, 1)
    with pytest.raises(zx.SimError):
        zx.sim_raw_add((2 ** 126, 0, 0, 0), (2 ** 126, 0, 0, 0))


def test_null_arguments_are_rejected():
    lib = binding.lib()
    assert lib.sim_ir_info(None, 0, None) == binding.SIM_EINVAL
    assert lib.sim_program_info(None, None) == binding.SIM_EINVAL
    out = binding.sim_zomega()
    assert lib.sim_eval_amplitude(None, None, ctypes.byref(out)) == binding.SIM_EINVAL
    assert b"null" in lib.sim_last_error()


def test_node_pairs_with_constant_product_are_folded():
    # (1 + w^{2 + 4l})(1 + w^{6 + 4l}) = 2 for every l (the node cancellation of Section 5):
    # the pair leaves the packed program; 1 + w^{4l} with 1 + w^{4 + 4l} makes it zero; a pair
    # whose product does depend on l stays
    from workloads.programs import ProgramSpec
    pr = ProgramSpec(4)
    f = pr.add_form(0, 0b0111)
    g = pr.add_form(1, 0b0111)  # the complement of f
    h = pr.add_form(0, 0b1010)
    pr.nodes += [(f, 2, 4), (f, 6, 4), (g, 1, 4), (f, 5, 4), (h, 3, 4)]
    info = zx.sim_ir_info(pr.to_text())
    assert info["n_factors"] == 3 and not info["is_zero"]
    pr2 = ProgramSpec(3)
    f2 = pr2.add_form(0, 0b011)
    pr2.nodes += [(f2, 0, 4), (f2, 4, 4), (pr2.add_form(0, 0b100), 1, 4)]
    assert zx.sim_ir_info(pr2.to_text())["is_zero"] == 1


def test_weight4_phase_parts_share_one_form():
    # w^(4 f) parts of linear terms on k forms take one combined form: the program keeps the
    # node forms, the forms with a coefficient mod 4, and at most one more
    p = 12
    prog = wl.ProgramSpec(p)
    for i in range(3):
        f = prog.add_form(i & 1, 0b111 << i)
        prog.nodes.append((f, 1, 2))
    four = [prog.add_form(i & 1, (0b1011 << i) & 0xFFF) for i in range(5)]
    prog.lin += [(4, f) for f in four]
    odd = prog.add_form(1, 0b110000000001)
    prog.lin.append((6, odd))
    assert zx.sim_ir_info(prog.to_text())["n_forms"] == 3 + 1 + 1
    # parts that add up to the constant 1 (-1 overall), to another term's form or to a node
    # factor's form leave no form of their own
    for case in ("constant", "opposite", "node"):
        prog = wl.weight4_phase_program(0, 10, 2, case)
        # (factors that can vanish kept: solved for, their forms would fold away too)
        n_forms = zx.sim_ir_info_flags(prog.to_text(), binding.SIM_IR_KEEP_VANISHING)["n_forms"]
        assert n_forms == len(prog.forms) - {"constant": 3, "opposite": 1, "node": 2}[case]


def _single_parameter_nodes(n_nodes, seed):
    rng = wl.SplitMix64(770, seed)
    prog = wl.ProgramSpec(n_nodes)
    for i in range(n_nodes):
        prog.nodes.append((prog.add_form(0, 1 << i), 0, 2))
    for _ in range(12):
        prog.lin.append((rng.randint(1, 7), prog.add_form(rng.randint(0, 1), rng.randint(1, (1 << n_nodes) - 1))))
    return prog


def test_block_sums_in_32_bits_stop_at_the_bound():
    # two form words, 64-term blocks: with 24 node factors a block's terms sum below 2^31
    # (24 + 6 <= 30) and are added in 32 bits (4 lane operations per term instead of 12, plus
    # 12 per block); with 25 they are not
    a = zx.sim_ir_info(_single_parameter_nodes(24, 24).to_text())
    b = zx.sim_ir_info(_single_parameter_nodes(25, 25).to_text())
    assert a["n_forms"] > 32 and b["n_forms"] > 32 and a["n_forms"] <= 64 and b["n_forms"] <= 64
    # (the one more high parameter adds 4 / 256 to the per-slice set-up)
    assert b["ops_per_term"] - a["ops_per_term"] == pytest.approx(8 - 12 / 64 + 4 / 256, abs=1e-9)


@pytest.mark.parametrize("n_nodes", [24, 25])
def test_int32_block_sums_would_wrap_past_the_bound(o2, n_nodes):
    # the block-sum bound program: a 64-term block of the low parameters sums to exactly
    # 2^(n+6) in one coordinate (oracle), which int32 holds at n = 24 and not at n = 25, where
    # 32-bit addition of the block's terms wraps to -2^31; the header enables 32-bit block sums
    # exactly where they cannot wrap
    import numpy as np
    text = wl.block_bound_program(n_nodes).to_text()
    block = o2.evaluate(text, first=0, count=64, terms=True)
    assert block["raw"] == (1 << (n_nodes + 6), 0, 0, 0)
    assert sorted(block["terms"]) == list(range(64))
    lanes = np.array([block["terms"][t][0] for t in range(64)], dtype=np.int64)
    assert (lanes == 1 << n_nodes).all()
    wrapped = int(lanes.astype(np.int32).sum(dtype=np.int32))
    fits = n_nodes + 6 <= 30
    assert (wrapped == 1 << (n_nodes + 6)) == fits
    if not fits:
        assert wrapped == -(1 << 31)
    assert zx.sim_ir_info(text)["block_sum32"] == (1 if fits else 0)
