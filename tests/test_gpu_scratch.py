"""Entry points with caller-owned device scratch (needs an MI355X): the *_ws calls, the
prepared batch enqueued without waiting (also replayed from a captured hipGraph) and the
shard ranges of sim_eval_range_ws.  Every value is compared exactly with the library-scratch
call it mirrors, and those with the oracle."""

import sys

import pytest

import paper_2403_06777_amd as zx
import workloads as wl

pytestmark = pytest.mark.gpu


def say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def _texts():
    texts = []
    for i in range(8):
        p = [3, 7, 12, 16, 18, 0, 9, 14][i]
        texts.append(wl.random_program(60 + i, p, n_nodes=10 + i, n_pairs=i % 3, n_lin=3 + (60 if i == 4 else 0),
                                       n_mono=(2 * p if i % 2 else 0), scalar_range=2).to_text())
    texts.append(wl.kernel_sized_program(2, p=22, n_factors=40, n_monomials=80).to_text())
    # a program of 2^27 terms: its own resident-grid launch inside the batch
    big, _ = wl.block_separable_program(5, 27, factors_per_block=2, lin_per_block=1)
    texts.append(big.to_text())
    zero = wl.ProgramSpec(4)
    zero.nodes = [(zero.add_form(1, 0), 0, 4)]
    texts.append(zero.to_text())
    return texts


@pytest.fixture(scope="module")
def programs(o2):
    import torch
    torch.cuda.init()
    texts = _texts()
    hs = [zx.sim_program_from_ir(t) for t in texts]
    want = [zx.sim_eval_amplitude(h) for h in hs]
    for t, w, h in zip(texts, want, hs):
        if zx.sim_program_info(h)["n_params"] <= 22:
            assert w == o2.evaluate(t)["canonical"]
    yield hs, want
    for h in hs:
        zx.sim_program_free(h)


def _scratch(nbytes):
    import torch
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def test_scratch_variants_equal_library_scratch(programs):
    hs, want = programs
    need = zx.sim_scratch_bytes(hs)
    say("scratch bytes", need)
    assert need > 0
    buf = _scratch(need)
    for h, w in zip(hs, want):
        assert zx.sim_eval_amplitude_ws(h, buf.data_ptr(), need) == w
    assert zx.sim_eval_batch_ws(hs, buf.data_ptr(), need) == want
    # the need depends on the tuning (smaller work items: more partials)
    t = {"chunk_log2": 12}
    need_t = zx.sim_scratch_bytes(hs, t)
    assert need_t > need
    with pytest.raises(zx.SimError):
        zx.sim_eval_batch_ws(hs, buf.data_ptr(), need, tuning=t)
    buf_t = _scratch(need_t)
    assert zx.sim_eval_batch_ws(hs, buf_t.data_ptr(), need_t, tuning=t) == want


def test_scratch_too_small_is_an_error(programs):
    hs, want = programs
    need = zx.sim_scratch_bytes(hs)
    buf = _scratch(need)
    with pytest.raises(zx.SimError) as e:
        zx.sim_eval_batch_ws(hs, buf.data_ptr(), 1024)
    assert e.value.code == zx.binding.SIM_ERANGE
    with pytest.raises(zx.SimError) as e:
        zx.sim_eval_amplitude_ws(hs[-2], buf.data_ptr(), 256)
    assert e.value.code == zx.binding.SIM_ERANGE
    with pytest.raises(zx.SimError) as e:  # misaligned
        zx.sim_eval_amplitude_ws(hs[0], buf.data_ptr() + 8, need - 8)
    assert e.value.code == zx.binding.SIM_EINVAL
    # the failed calls left nothing behind
    assert zx.sim_eval_batch_ws(hs, buf.data_ptr(), need) == want


def test_shard_ranges_add_to_the_whole(programs):
    hs, want = programs
    need = zx.sim_scratch_bytes(hs)
    buf = _scratch(need)
    for h in hs[-3:-1]:
        info = zx.sim_program_info(h)
        p, wb = info["n_params"], info["walk_bits"]
        whole = zx.sim_eval_range(h, 0, info["n_slices"])
        for g in sorted({wb, min(p, wb + 3), p}):
            n = 1 << (p - g)
            total = (0, 0, 0, 0)
            for k in range(n):
                total = zx.sim_raw_add(total, zx.sim_eval_range_ws(h, k, 1, g, buf.data_ptr(), need))
            say("shards", p, g, n)
            assert total == whole
        assert zx.sim_finalize(h, whole) == want[hs.index(h)]
        with pytest.raises(zx.SimError):
            zx.sim_eval_range_ws(h, 0, 1, wb - 1 if wb else p + 1, buf.data_ptr(), need)
        with pytest.raises(zx.SimError):
            zx.sim_eval_range_ws(h, 1, 1 << (p - wb), wb, buf.data_ptr(), need)


def test_enqueued_batch_replays_from_a_captured_graph(programs):
    import torch
    hs, want = programs
    n = len(hs)
    need = zx.sim_scratch_bytes(hs)
    buf = _scratch(need)
    out = torch.zeros(72 * n, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    zx.sim_batch_prepare(hs, buf.data_ptr(), need, s)
    # eager enqueue first
    zx.sim_enqueue_batch(hs, buf.data_ptr(), need, out.data_ptr(), s)
    torch.cuda.synchronize()
    assert zx.zomegas_from_bytes(out.cpu().numpy().tobytes(), n) == want
    # captured once, replayed with eager library work and synchronisations between replays
    g = torch.cuda.CUDAGraph()
    out.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        zx.sim_enqueue_batch(hs, buf.data_ptr(), need, out.data_ptr(), s)
    for rep in range(4):
        say("graph replay", rep)
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert zx.zomegas_from_bytes(out.cpu().numpy().tobytes(), n) == want
        assert zx.sim_eval_amplitude(hs[rep]) == want[rep]
        assert zx.sim_eval_batch(hs[:3]) == want[:3]
    del g
    zx.sim_batch_forget(buf.data_ptr())


def test_enqueued_amplitudes_replay_from_a_captured_graph(programs):
    # the documented recipe: after evaluations enqueued on another stream, one call on the
    # capture stream (which waits for them), then the capture; every replay, with synchronous
    # library calls between replays, writes the synchronous values
    import torch
    hs, want = programs
    n = len(hs)
    out = torch.zeros(72 * n, dtype=torch.uint8, device="cuda")
    s0, s = torch.cuda.Stream(), torch.cuda.Stream()
    for k, h in enumerate(hs):
        zx.sim_enqueue_amplitude(h, out.data_ptr() + 72 * k, s0)
    zx.sim_enqueue_amplitude(hs[0], out.data_ptr(), s)
    torch.cuda.synchronize()
    assert zx.zomegas_from_bytes(out.cpu().numpy().tobytes(), n) == want
    # the capture holds the programs with a value (a zero program's result is a host copy)
    keep = [k for k in range(n) if not zx.sim_program_info(hs[k])["is_zero"]]
    hs, want, n = [hs[k] for k in keep], [want[k] for k in keep], len(keep)
    assert n >= 5
    g = torch.cuda.CUDAGraph()
    out.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        for k, h in enumerate(hs):
            zx.sim_enqueue_amplitude(h, out.data_ptr() + 72 * k, s)
    for rep in range(4):
        say("amplitude graph replay", rep)
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert zx.zomegas_from_bytes(out.cpu().numpy().tobytes(), n) == want
        assert zx.sim_eval_amplitude(hs[rep % n]) == want[rep % n]
        if rep == 1:
            # a large batch may outgrow the library's scratch: the graph keeps the buffer it was
            # captured with, which the library does not free
            assert zx.sim_eval_batch(hs * 40) == want * 40
    del g


def test_enqueue_needs_a_prepared_region(programs):
    import torch
    hs, want = programs
    need = zx.sim_scratch_bytes(hs)
    buf = _scratch(need)
    out = torch.zeros(72 * len(hs), dtype=torch.uint8, device="cuda")
    zx.sim_batch_forget(buf.data_ptr())
    with pytest.raises(zx.SimError) as e:
        zx.sim_enqueue_batch(hs, buf.data_ptr(), need, out.data_ptr())
    assert e.value.code == zx.binding.SIM_EINVAL
    zx.sim_batch_prepare(hs[:4], buf.data_ptr(), need)
    with pytest.raises(zx.SimError):  # prepared for other programs
        zx.sim_enqueue_batch(hs, buf.data_ptr(), need, out.data_ptr())
    zx.sim_enqueue_batch(hs[:4], buf.data_ptr(), need, out.data_ptr())
    torch.cuda.synchronize()
    assert zx.zomegas_from_bytes(out.cpu().numpy().tobytes(), 4) == want[:4]
    zx.sim_batch_forget(buf.data_ptr())
