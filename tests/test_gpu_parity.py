"""Parity of the HIP path with the oracle, through the C-ABI (needs an MI355X).

Every expected value comes from the oracle (term-by-term evaluator) or from a closed form
built from oracle results; the comparison is exact equality of canonical Z[w] scalars.
"""

import sys

import pytest

import paper_2403_06777_amd as zx
import workloads as wl
from oracle import zomega as zw

pytestmark = pytest.mark.gpu


def say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def gpu_value(text, flags=0):
    h = zx.sim_program_from_ir_flags(text, flags)
    try:
        return zx.sim_eval_amplitude(h)
    finally:
        zx.sim_program_free(h)


def oracle_value(o2, text):
    return o2.evaluate(text)["canonical"]


@pytest.mark.parametrize("p,factors,monos", [(4, 8, 10), (9, 16, 30), (13, 32, 60), (17, 64, 120), (20, 64, 200)])
def test_kernel_sized_family_exhaustive(o2, p, factors, monos):
    for seed in range(2):
        prog = wl.kernel_sized_program(seed, p=p, n_factors=factors, n_monomials=monos)
        text = prog.to_text()
        say("kernel-sized family", p, factors, monos, seed)
        assert gpu_value(text) == oracle_value(o2, text)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 5, 8, 11, 14, 18])
def test_random_programs_exhaustive(o2, p):
    for seed in range(3):
        prog = wl.random_program(seed, p, n_nodes=12, n_pairs=2 if p else 0, n_lin=6, n_mono=3 * p,
                                 scalar_range=3, shared_forms=bool(seed % 2))
        text = prog.to_text()
        say("random program", p, seed)
        assert gpu_value(text) == oracle_value(o2, text)


@pytest.mark.parametrize("n_lin,p", [(80, 12), (200, 14), (420, 10)])
def test_wide_form_vectors(o2, n_lin, p):
    # more than 64, 128 and 256 forms: W = 4, 8 and 16 words per lane
    prog = wl.random_program(7, p, n_nodes=30, n_lin=n_lin, n_mono=10, scalar_range=2)
    text = prog.to_text()
    info = zx.sim_ir_info(text)
    say("wide forms", info["n_forms"])
    assert gpu_value(text) == oracle_value(o2, text)


def test_appendix_d_example_total():
    total = None
    for t in wl.appendix_d_terms():
        (c, e) = gpu_value(t.to_text())
        total = (c, e) if total is None else zw.add_scalar(*total, c, e)
    assert total == zw.canonical((80, 0, 16, 0), 0)


def test_zero_and_constant_programs(o2):
    prog = wl.ProgramSpec(5)
    f = prog.add_form(0, 0)
    prog.nodes = [(f, 4, 0)]
    assert gpu_value(prog.to_text()) == ((0, 0, 0, 0), 0)
    prog = wl.ProgramSpec(0)
    prog.scalar = (3, -1, 2, 0)
    prog.sqrt2_exp = -3
    text = prog.to_text()
    assert gpu_value(text) == oracle_value(o2, text)


@pytest.mark.parametrize("p,fpb", [(24, 3), (32, 4), (36, 6)])
def test_closed_form_block_programs(o2, p, fpb):
    # scrambled block-separable programs: the sum is the product of the block sums
    full, blocks = wl.block_separable_program(p, p, factors_per_block=fpb, lin_per_block=2,
                                              pairs_per_block=1 if p < 36 else 0, scramble=True)
    expect = zw.ONE
    for blk in blocks:
        expect = zw.mul(expect, o2.evaluate(blk.to_text(), threads=1)["raw"])
    say("closed form", p, fpb, "log2|expect|", max(abs(v) for v in expect).bit_length())
    assert gpu_value(full.to_text()) == zw.canonical(expect, 0)


def test_closed_form_with_monomials(o2):
    full, blocks = wl.block_separable_program(5, 32, factors_per_block=3, lin_per_block=1, mono_per_block=3,
                                              scramble=False)
    expect = zw.ONE
    for blk in blocks:
        expect = zw.mul(expect, o2.evaluate(blk.to_text(), threads=1)["raw"])
    say("closed form with monomials")
    assert gpu_value(full.to_text()) == zw.canonical(expect, 0)


def test_folded_node_pairs_keep_the_sum(o2):
    # random programs with planted node pairs whose product is constant (some on complemented
    # forms, some making the program zero): the packed program, without them, has the sum of
    # the program as written
    from workloads.programs import ProgramSpec
    for seed in range(8):
        prog = wl.random_program(seed, 12, n_nodes=10, n_lin=6, n_mono=12)
        rng = wl.SplitMix64(79, seed)
        for _ in range(3):
            f = rng.randint(0, len(prog.forms) - 1)
            cst, mask = prog.forms[f]
            g = prog.add_form(1 - cst, mask)
            a = rng.choice([1, 2, 3, 5, 6, 7]) if seed % 4 else rng.choice([0, 4])
            prog.nodes += [(f, a, 4), (g, a, 4)]  # values swapped: product constant
        text = prog.to_text()
        say("folded node pairs", seed, zx.sim_ir_info(text)["n_factors"], len(prog.nodes))
        assert gpu_value(text) == oracle_value(o2, text)


KEEP = zx.binding.SIM_IR_KEEP_VANISHING


def test_vanishing_step_table_and_basis_paths(o2):
    # factors that can vanish kept at run time (SIM_IR_KEEP_VANISHING; by default they are
    # solved for exactly): a block's surviving steps come from the hashed table when the
    # vanishing bits lie in word 0 (kernel-sized programs), else from the reduced-basis test
    # (more than 32 vanishing factors); both against the oracle, exhaustively at p = 20 and 24,
    # and on sampled slices of two p = 32 programs
    from tests.test_abi_cpu import wide_vanishing_program
    for seed in range(4):
        text = wl.kernel_sized_program(seed, p=20, n_factors=64, n_monomials=200).to_text()
        assert zx.sim_ir_info_flags(text, KEEP)["vanish_table_bits"] > 0
        say("vanishing steps, table", seed)
        assert gpu_value(text, KEEP) == oracle_value(o2, text)
    for seed in range(3):
        text = wide_vanishing_program(seed).to_text()
        info = zx.sim_ir_info_flags(text, KEEP)
        assert info["vanish_table_bits"] == 0 and info["nonzero_fraction"] > 0
        say("vanishing steps, basis", seed, info["nonzero_fraction"])
        assert gpu_value(text, KEEP) == oracle_value(o2, text)
    for seed in (1, 3):
        text = wl.kernel_sized_program(seed).to_text()
        h = zx.sim_program_from_ir_flags(text, KEEP)
        try:
            info = zx.sim_program_info(h)
            assert info["vanish_table_bits"] > 0
            perm = zx.sim_program_layout(h)
            wb, ns = info["walk_bits"], info["n_slices"]
            rng = wl.SplitMix64(78, seed)
            for _ in range(3):
                s0 = rng.randint(0, ns - 16)
                say("vanishing steps p32", seed, s0)
                ref = o2.evaluate(text, first=s0 << wb, count=16 << wb, perm=perm)["raw"]
                assert zx.sim_eval_range(h, s0, 16) == ref
        finally:
            zx.sim_program_free(h)


def test_kernel_sized_full_size_sampled_slices(o2):
    # p = 32 (2^21 surviving terms after the exact elimination): the whole sum equals the sum of
    # range partials, and sampled ranges equal the oracle on exactly the same assignments (the
    # points of the surviving subspace that the slices cover; compared finalised, since the
    # vanishing factors, constant on the subspace, are in the packed constant)
    prog = wl.kernel_sized_program(0)
    text = prog.to_text()
    h = zx.sim_program_from_ir(text)
    try:
        info = zx.sim_program_info(h)
        x0, cols = zx.sim_program_affine_layout(h)
        wb, ns = info["walk_bits"], info["n_slices"]
        say("full size", info)
        assert info["n_eliminated"] == 11 and info["n_params"] == 21
        whole = zx.sim_eval_amplitude(h)
        parts = (0, 0, 0, 0)
        G = 8
        for g in range(G):
            a, b = g * ns // G, (g + 1) * ns // G
            parts = zx.sim_raw_add(parts, zx.sim_eval_range(h, a, b - a))
        assert zx.sim_finalize(h, parts) == whole
        rng = wl.SplitMix64(77, 0)
        for _ in range(4):
            s0 = rng.randint(0, ns - 16)
            raw = zx.sim_eval_range(h, s0, 16)
            ref = o2.evaluate(text, first=s0 << wb, count=16 << wb, points=(x0, cols))["canonical"]
            say("slices", s0, raw, ref)
            assert zx.sim_finalize(h, raw) == ref
    finally:
        zx.sim_program_free(h)


def test_range_partials_match_oracle_ranges(o2):
    prog = wl.random_program(3, 16, n_nodes=20, n_pairs=2, n_lin=5, n_mono=30, scalar_range=2)
    text = prog.to_text()
    h = zx.sim_program_from_ir(text)
    try:
        info = zx.sim_program_info(h)
        perm = zx.sim_program_layout(h)
        wb, ns = info["walk_bits"], info["n_slices"]
        for s0, n in [(0, 1), (3, 5), (ns - 7, 7), (0, ns)]:
            raw = zx.sim_eval_range(h, s0, n)
            ref = o2.evaluate(text, first=s0 << wb, count=n << wb, perm=perm)["raw"]
            assert raw == ref
        assert zx.sim_eval_range(h, 5, 0) == (0, 0, 0, 0)
        with pytest.raises(zx.SimError):
            zx.sim_eval_range(h, ns, 1)
    finally:
        zx.sim_program_free(h)


def _batch_programs():
    progs = []
    for i in range(10):
        p = [3, 7, 12, 16, 18, 0, 9, 14, 20, 11][i]
        progs.append(wl.random_program(40 + i, p, n_nodes=10 + i, n_pairs=i % 3, n_lin=3 + (60 if i == 4 else 0),
                                       n_mono=(2 * p if i % 2 else 0), scalar_range=2))
    z = wl.ProgramSpec(4)
    f = z.add_form(1, 0)
    z.nodes = [(f, 0, 4)]
    progs.append(z)
    return [p.to_text() for p in progs]


def test_batch_equals_single_evaluations(o2):
    texts = _batch_programs()
    hs = [zx.sim_program_from_ir(t) for t in texts]
    try:
        single = [zx.sim_eval_amplitude(h) for h in hs]
        for t, s in zip(texts, single):
            assert s == oracle_value(o2, t)
        for tuning in (None, {"chunk_log2": 10}, {"chunk_log2": 14, "block_threads": 128, "blocks_per_cu": 2}):
            say("batch", tuning)
            assert zx.sim_eval_batch(hs, tuning=tuning) == single
        # batch of ranges
        infos = [zx.sim_program_info(h) for h in hs]
        firsts = [i["n_slices"] // 3 for i in infos]
        counts = [i["n_slices"] - f for f, i in zip(firsts, infos)]
        raws = zx.sim_eval_ranges(hs, firsts, counts)
        for h, f, c, r in zip(hs, firsts, counts, raws):
            assert r == zx.sim_eval_range(h, f, c)
    finally:
        for h in hs:
            zx.sim_program_free(h)


def test_batch_plan_graph_replays(o2):
    texts = _batch_programs()
    hs = [zx.sim_program_from_ir(t) for t in texts]
    plan = None
    try:
        single = [zx.sim_eval_amplitude(h) for h in hs]
        plan = zx.sim_batch_plan_create(hs, {"chunk_log2": 12})
        for rep in range(4):
            say("plan replay", rep)
            assert zx.sim_batch_plan_run(plan, len(hs)) == single
            # eager work between replays
            assert zx.sim_eval_amplitude(hs[rep]) == single[rep]
    finally:
        if plan:
            zx.sim_batch_plan_free(plan)
        for h in hs:
            zx.sim_program_free(h)


def test_torch_stream_is_accepted():
    import torch
    s = torch.cuda.Stream()
    prog = wl.kernel_sized_program(3, p=14, n_factors=20, n_monomials=30)
    h = zx.sim_program_from_ir(prog.to_text())
    try:
        assert zx.sim_eval_amplitude(h, s) == zx.sim_eval_amplitude(h)
        val, ms = zx.sim_eval_timed(h, s)
        assert val == zx.sim_eval_amplitude(h) and ms > 0
    finally:
        zx.sim_program_free(h)


def test_finalize_batch_matches_single_finalize():
    texts = _batch_programs()
    hs = [zx.sim_program_from_ir(t) for t in texts]
    try:
        raws = [zx.sim_eval_range(h, 0, zx.sim_program_info(h)["n_slices"]) for h in hs]
        assert zx.sim_finalize_batch(hs, raws) == [zx.sim_finalize(h, r) for h, r in zip(hs, raws)]
        assert zx.sim_finalize_batch(hs, raws) == [zx.sim_eval_amplitude(h) for h in hs]
    finally:
        for h in hs:
            zx.sim_program_free(h)


def test_batch_with_programs_above_the_own_launch_size(o2):
    # programs of 2^26 terms and more run as their own launches inside a batch and its captured
    # plan, beside the queued small ones; closed forms (oracle block sums) pin the large ones
    full, blocks = wl.block_separable_program(11, 28, factors_per_block=4, lin_per_block=2, pairs_per_block=1,
                                              scramble=True)
    expect_big = zw.ONE
    for blk in blocks:
        expect_big = zw.mul(expect_big, o2.evaluate(blk.to_text(), threads=1)["raw"])
    mono_full, mono_blocks = wl.block_separable_program(12, 32, factors_per_block=3, lin_per_block=1,
                                                        mono_per_block=3, scramble=False)
    expect_mono = zw.ONE
    for blk in mono_blocks:
        expect_mono = zw.mul(expect_mono, o2.evaluate(blk.to_text(), threads=1)["raw"])
    texts = [full.to_text()] + _batch_programs()[:5] + [mono_full.to_text()]
    hs = [zx.sim_program_from_ir(t) for t in texts]
    plan = None
    try:
        expect = [zw.canonical(expect_big, 0)] + [oracle_value(o2, t) for t in texts[1:6]] + \
                 [zw.canonical(expect_mono, 0)]
        say("large in batch")
        assert zx.sim_eval_batch(hs) == expect
        plan = zx.sim_batch_plan_create(hs, None)
        for rep in range(3):
            say("large in plan", rep)
            assert zx.sim_batch_plan_run(plan, len(hs)) == expect
            assert zx.sim_eval_amplitude(hs[1]) == expect[1]
        # ranges of the large program inside a batch equal its own range partials
        info = zx.sim_program_info(hs[0])
        ns = info["n_slices"]
        raws = zx.sim_eval_ranges([hs[0], hs[0]], [0, ns // 3], [ns // 3, ns - ns // 3])
        assert zx.sim_raw_add(raws[0], raws[1]) == zx.sim_eval_range(hs[0], 0, ns)
    finally:
        if plan:
            zx.sim_batch_plan_free(plan)
        for h in hs:
            zx.sim_program_free(h)


@pytest.mark.parametrize("n_nodes,n_lin,p", [(1, 3, 9), (5, 40, 14), (10, 100, 16), (7, 200, 13), (3, 0, 18)])
def test_node_table_programs(o2, n_nodes, n_lin, p):
    # at most 10 node factors (general a, b: some can vanish), linear phase terms sharing forms
    # with them, widths 1 to 8 words: the node factors come from the node table
    for seed in range(3):
        prog = wl.random_program(100 + seed, p, n_nodes=n_nodes, n_pairs=0, n_lin=n_lin, n_mono=p if seed == 2 else 0,
                                 scalar_range=2, shared_forms=bool(seed % 2))
        text = prog.to_text()
        say("node table", n_nodes, n_lin, p, seed, zx.sim_ir_info(text)["n_forms"])
        assert gpu_value(text) == oracle_value(o2, text)


def test_node_table_largest_terms(o2):
    # ten node factors 1 + w^0 = 2 at l = 0 (1 + w^2 at l = 1) on single parameters: terms up
    # to 2^10 in a coordinate, the most a node-table block sums in 32 bits; the linear terms
    # give the terms both signs
    for seed in range(2):
        rng = wl.SplitMix64(760, seed)
        p = 16
        prog = wl.ProgramSpec(p)
        for i in range(10):
            prog.nodes.append((prog.add_form(0, 1 << i), 0, 2))
        for _ in range(12):
            m = rng.randint(1, (1 << p) - 1)
            prog.lin.append((rng.randint(1, 7), prog.add_form(rng.randint(0, 1), m)))
        text = prog.to_text()
        say("largest node-table terms", seed)
        assert gpu_value(text) == oracle_value(o2, text)


@pytest.mark.parametrize("n_nodes", [24, 25])
def test_block_sums_at_the_int32_bound(o2, n_nodes):
    # 24 node factors 1 + w^0 = 2 at l = 0 on single parameters, two form words (64-term
    # blocks): terms up to 2^24 in a coordinate, 64 of them just below 2^31, the most a block
    # sums in 32 bits; with 25 factors the block sums stay in int64
    rng = wl.SplitMix64(770, n_nodes)
    p = n_nodes
    prog = wl.ProgramSpec(p)
    for i in range(n_nodes):
        prog.nodes.append((prog.add_form(0, 1 << i), 0, 2))
    for _ in range(12):
        prog.lin.append((rng.randint(1, 7), prog.add_form(rng.randint(0, 1), rng.randint(1, (1 << p) - 1))))
    text = prog.to_text()
    say("int32 block-sum bound", n_nodes, zx.sim_ir_info(text)["n_forms"])
    assert gpu_value(text) == oracle_value(o2, text)


@pytest.mark.parametrize("n_nodes", [24, 25])
def test_block_sums_reach_the_int32_bound(o2, n_nodes):
    # every node factor 1 + w^l on the one top parameter (a slice bit): in a slice with it 0 each
    # of a 64-term block's terms is exactly 2^n times a phase that is the same across the block
    # (linear terms on slice bits only, which also make two form words), so with 24 factors a
    # block sums to 2^30 in a coordinate, the most that 32-bit block sums take; with 25 (2^31,
    # which int32 cannot hold) the header leaves them off
    p = 14
    text = wl.block_bound_program(n_nodes, p).to_text()
    info = zx.sim_ir_info(text)
    assert info["n_forms"] > 32 and info["walk_bits"] <= p - 6
    assert info["block_sum32"] == (1 if n_nodes == 24 else 0)
    say("int32 block sums at 2^30 / 2^31", n_nodes)
    assert gpu_value(text) == oracle_value(o2, text)


@pytest.mark.parametrize("case", ["random", "node", "opposite", "constant"])
def test_weight4_phase_parts_combined(o2, case):
    # the weight-4 parts of the linear phase terms as one form: beside node tables of 1 to 10
    # factors (the combined bit makes 11 table bits at 10 factors), with 20 or 31 factors
    # (R*4 slot read from word 0 beside wider form vectors), on a node factor's form, on
    # another term's form with the other constant, or adding up to a constant
    for n_nodes, p in [(1, 9), (4, 13), (10, 15), (0, 11), (6, 22), (20, 16), (31, 14)]:
        if case == "node" and n_nodes == 0:
            continue
        prog = wl.weight4_phase_program(n_nodes, p, n_nodes, case)
        text = prog.to_text()
        say("weight-4 parts", case, n_nodes, p, zx.sim_ir_info(text)["n_forms"])
        assert gpu_value(text) == oracle_value(o2, text), (case, n_nodes, p)


def test_enqueued_evaluations_match_synchronous_ones(o2):
    # several programs enqueued back to back (one stream, then two streams, then mixed with
    # synchronous calls that reuse the device's scratch): every device-written value equals the
    # synchronous one; a zero program writes zero
    import torch
    texts = [wl.kernel_sized_program(seed, p=18 + seed, n_factors=32, n_monomials=60).to_text() for seed in range(4)]
    texts.append(wl.random_program(5, 10, n_nodes=0, n_lin=4).to_text())
    zero = ProgramSpecZero()
    hs = [zx.sim_program_from_ir(t) for t in texts + [zero]]
    try:
        want = [zx.sim_eval_amplitude(h) for h in hs]
        assert want[-1] == ((0, 0, 0, 0), 0)
        say("enqueue", [zx.sim_program_info(h)["n_params"] for h in hs])
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        for streams in ([s1], [s1, s2]):
            out = torch.zeros(72 * len(hs) * 2, dtype=torch.uint8, device="cuda")
            for k in range(2 * len(hs)):
                zx.sim_enqueue_amplitude(hs[k % len(hs)], out.data_ptr() + 72 * k, streams[k % len(streams)])
                if k == 3:  # a synchronous call in between waits for the enqueued work
                    assert zx.sim_eval_amplitude(hs[1]) == want[1]
            torch.cuda.synchronize()
            host = out.cpu().numpy().tobytes()
            got = [zx.zomega_from_bytes(host[72 * k:72 * (k + 1)]) for k in range(2 * len(hs))]
            assert got == want + want
    finally:
        for h in hs:
            zx.sim_program_free(h)


def ProgramSpecZero():
    # 1 + w^4 as a constant factor: the program is zero
    from workloads.programs import ProgramSpec
    pr = ProgramSpec(6)
    f = pr.add_form(1, 0)
    pr.nodes.append((f, 0, 4))
    pr.nodes.append((pr.add_form(0, 0b101), 1, 4))
    return pr.to_text()


def _aligned_blocks(seed, p, fpb):
    # blocks of 4 parameters whose factors 1 + w^(2 l) are 2 or 1 + i (no linear phases): the
    # block sums do not cancel, so the whole sum exceeds 2^64 (int128 sums); relabelled by a
    # random invertible affine map, which keeps the sum
    from workloads.programs import ProgramSpec, _random_invertible_rows, _parity
    rng = wl.SplitMix64(85, seed)
    full, blocks = ProgramSpec(p), []
    for off in range(0, p, 4):
        blk = ProgramSpec(4)
        for _ in range(fpb):
            blk.nodes.append((blk.add_form(rng.randint(0, 1), rng.randint(1, 15)), 0, 2))
        blocks.append(blk)
        base = len(full.forms)
        full.forms += [(c, m << off) for c, m in blk.forms]
        full.nodes += [(base + f, a, b) for f, a, b in blk.nodes]
    rows = _random_invertible_rows(rng, p)
    shift = rng.randint(0, (1 << p) - 1)
    forms = []
    for c, m in full.forms:
        mm = 0
        for i in range(p):
            if m >> i & 1:
                mm ^= rows[i]
        forms.append((c ^ _parity(m & shift), mm))
    full.forms = forms
    return full, blocks


@pytest.mark.parametrize("p,fpb", [(40, 4), (44, 3)])
def test_closed_forms_int128_stress(o2, p, fpb):
    full, blocks = _aligned_blocks(p, p, fpb)
    expect = zw.ONE
    for blk in blocks:
        expect = zw.mul(expect, o2.evaluate(blk.to_text(), threads=1)["raw"])
    bits = max(abs(v) for v in expect).bit_length()
    info = zx.sim_ir_info(full.to_text())
    say("int128 stress", p, fpb, "log2|sum|", bits, "ops/term", info["ops_per_term"])
    assert bits > 64 and info["n_params"] == p
    assert gpu_value(full.to_text()) == zw.canonical(expect, 0)
