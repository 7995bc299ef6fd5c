"""The allocation-free entry point (sim_eval_ranges_static) against the entry point it mirrors
(sim_eval_ranges), exactly, on two calls in a row with a smaller batch the second time; a
batch that needs more than the fixed array is refused (needs an MI355X)."""

import sys

import pytest

import paper_2403_06777_amd as zx
import workloads as wl

pytestmark = pytest.mark.gpu


def say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def _programs():
    texts = []
    for i in range(9):
        p = [5, 9, 12, 16, 19, 0, 11, 14, 22][i]
        texts.append(wl.random_program(90 + i, p, n_nodes=8 + i, n_pairs=i % 3, n_lin=4, n_mono=(2 * p if i % 2 else 0),
                                       scalar_range=2).to_text())
    texts.append(wl.kernel_sized_program(4, p=24, n_factors=48, n_monomials=100).to_text())
    big, _ = wl.block_separable_program(9, 27, factors_per_block=2, lin_per_block=1)
    texts.append(big.to_text())
    return texts


def test_static_ranges_equal_ranges(o2):
    hs = [zx.sim_program_from_ir(t) for t in _programs()]
    try:
        infos = [zx.sim_program_info(h) for h in hs]
        # first call: every program, the last two thirds of its slices
        firsts = [i["n_slices"] // 3 for i in infos]
        counts = [i["n_slices"] - f for f, i in zip(firsts, infos)]
        say("static ranges, call 1", len(hs))
        want = zx.sim_eval_ranges(hs, firsts, counts)
        assert zx.sim_eval_ranges_static(hs, firsts, counts) == want
        # the small programs' ranges also match the oracle on the same assignments (a raw partial
        # leaves out the packed program's constant, which includes the constant factors folded at
        # packing, so the comparison is of finalised values)
        for h, i, f, c, w in zip(hs, infos, firsts, counts, want):
            if i["n_params"] <= 16 and i["n_slices"] > 1:
                points = zx.sim_program_affine_layout(h)
                t = zx.sim_program_ir(h)
                wb = i["walk_bits"]
                ref = o2.evaluate(t, first=f << wb, count=c << wb, points=points)["canonical"]
                assert zx.sim_finalize(h, w) == ref
        # second call: fewer programs, shorter ranges
        sub = [0, 3, 6]
        f2 = [1 for _ in sub]
        c2 = [max(0, infos[k]["n_slices"] - 2) for k in sub]
        say("static ranges, call 2", len(sub))
        want2 = zx.sim_eval_ranges([hs[k] for k in sub], f2, c2)
        assert zx.sim_eval_ranges_static([hs[k] for k in sub], f2, c2) == want2
        # whole programs finalise to the single evaluation
        whole = zx.sim_eval_ranges_static(hs, [0] * len(hs), [i["n_slices"] for i in infos])
        for h, r in zip(hs, whole):
            assert zx.sim_finalize(h, r) == zx.sim_eval_amplitude(h)
    finally:
        for h in hs:
            zx.sim_program_free(h)


def test_static_ranges_refuse_what_does_not_fit():
    # 40 programs of 2^25 terms (their vanishing factors kept, so nothing is solved for) in work
    # items of 2^13 terms: 4096 items each, whose partials and layout (about 14 MB) exceed the
    # fixed array
    prog = wl.kernel_sized_program(6, p=25, n_factors=20, n_monomials=0)
    h = zx.sim_program_from_ir_flags(prog.to_text(), zx.binding.SIM_IR_KEEP_VANISHING)
    try:
        info = zx.sim_program_info(h)
        with pytest.raises(zx.SimError) as e:
            zx.sim_eval_ranges_static([h] * 40, [0] * 40, [info["n_slices"]] * 40, tuning={"chunk_log2": 13})
        assert e.value.code == zx.binding.SIM_ERANGE
        # a batch that fits still works after the refusal
        r = zx.sim_eval_ranges_static([h], [0], [info["n_slices"]])
        assert zx.sim_finalize(h, r[0]) == zx.sim_eval_amplitude(h)
    finally:
        zx.sim_program_free(h)
