"""Continuous batching on the GPU: every request's result in the mix is identical to its
solo evaluation (tolerance 0), and equal to the one-launch-per-query baseline."""

import pytest

import paper_2403_06777_amd as zx
import paper_2403_06777_amd.serving as S
import workloads as wl

pytestmark = pytest.mark.gpu


def test_serve_step_carries_and_finalises(o2):
    # three ticks over two programs of uneven size: the carried raw sums and the finalisation
    # in the last step give the single evaluation, which equals the oracle
    texts = [wl.kernel_sized_program(5, p=18, n_factors=30, n_monomials=60).to_text(),
             wl.random_program(6, 14, n_nodes=12, n_pairs=1, n_lin=4, n_mono=20, scalar_range=2).to_text()]
    hs = [zx.sim_program_from_ir(t) for t in texts]
    try:
        want = [zx.sim_eval_amplitude(h) for h in hs]
        assert want == [o2.evaluate(t)["canonical"] for t in texts]
        ns = [zx.sim_program_info(h)["n_slices"] for h in hs]
        cuts = [[0, n // 3, n // 2, n] for n in ns]
        carry = [(0, 0, 0, 0), (0, 0, 0, 0)]
        for k in range(3):
            firsts = [c[k] for c in cuts]
            counts = [c[k + 1] - c[k] for c in cuts]
            last = [k == 2, k == 2]
            out = zx.sim_serve_step(hs, firsts, counts, carry, last)
            if k < 2:
                carry = out
        assert out == want
    finally:
        for h in hs:
            zx.sim_program_free(h)


def test_pipelined_steps_carry_on_the_device(o2):
    # three steps enqueued back to back without waiting (device-resident carried sums in slots
    # 5 and 2 of 8), a third program finished in one step; results equal the single evaluations
    import torch
    texts = [wl.kernel_sized_program(5, p=18, n_factors=30, n_monomials=60).to_text(),
             wl.random_program(6, 14, n_nodes=12, n_pairs=1, n_lin=4, n_mono=20, scalar_range=2).to_text(),
             wl.kernel_sized_program(7, p=12, n_factors=20, n_monomials=30).to_text()]
    hs = [zx.sim_program_from_ir(t) for t in texts]
    try:
        want = [zx.sim_eval_amplitude(h) for h in hs]
        ns = [zx.sim_program_info(h)["n_slices"] for h in hs[:2]]
        cuts = [[0, n // 3, n // 2, n] for n in ns]
        carry = torch.zeros(8 * 72, dtype=torch.uint8, device="cuda")
        outs = [torch.zeros(3 * 72, dtype=torch.uint8, device="cuda") for _ in range(3)]
        s = torch.cuda.current_stream()
        for k in range(3):
            progs = hs[:2] + ([hs[2]] if k == 1 else [])
            firsts = [c[k] for c in cuts] + ([0] if k == 1 else [])
            counts = [c[k + 1] - c[k] for c in cuts] + ([zx.sim_program_info(hs[2])["n_slices"]] if k == 1 else [])
            flags = [(1 if k == 0 else 0) | (2 if k == 2 else 0)] * 2 + ([3] if k == 1 else [])
            zx.sim_serve_enqueue(progs, firsts, counts, [5, 2] + ([0] if k == 1 else []), flags, carry.data_ptr(), 8,
                                 outs[k].data_ptr(), s)
        torch.cuda.synchronize()
        last = zx.zomegas_from_bytes(outs[2].cpu().numpy().tobytes(), 2)
        assert last == want[:2]
        assert zx.zomegas_from_bytes(outs[1].cpu().numpy().tobytes(), 3)[2] == want[2]
        with pytest.raises(zx.SimError):  # one slot twice in a step
            zx.sim_serve_enqueue(hs[:2], [0, 0], [1, 1], [3, 3], [1, 1], carry.data_ptr(), 8, outs[0].data_ptr(), s)
    finally:
        for h in hs:
            zx.sim_program_free(h)


def test_served_results_equal_the_oracle(o2):
    # every served request whose compiled program has at most 22 parameters, against the
    # oracle's evaluation of the same compiled program (its IR text)
    pool = wl.serving_pool(10)
    reqs = S.make_stream(pool, 50, rate=300.0, seed=8)
    backend = S.ZxBackend(p_cap=26)
    srv = S.Server(backend, mem_budget=64 << 20, max_active=32, tick_terms=1 << 20, compile_workers=4)
    try:
        st = srv.run(reqs, realtime=True)
    finally:
        srv.close()
    checked = 0
    for r in reqs:
        if r.status != "done" or r.p > 22:
            continue
        q = zx.amplitude_query(r.bits) if r.kind == "amplitude" else zx.marginal_query(r.n_qubits, r.qubit, r.value)
        ir, info = zx.sim_compile_to_ir(r.circuit, q, p_cap=26)
        assert info["n_params"] == r.p
        assert r.result == o2.evaluate(ir)["canonical"], r.rid
        checked += 1
    assert checked >= 20 and st.done + st.rejected == len(reqs)


def test_results_in_the_mix_equal_solo_results():
    pool = wl.serving_pool(12)
    reqs = S.make_stream(pool, 60, rate=400.0, seed=3)
    backend = S.ZxBackend(p_cap=26)
    srv = S.Server(backend, mem_budget=64 << 20, max_active=32, tick_terms=1 << 22, compile_workers=4)
    try:
        st = srv.run(reqs, realtime=True)
    finally:
        srv.close()
    assert st.done + st.rejected == len(reqs)
    assert st.done > 20
    assert st.ticks < st.done * 64
    solo = {}
    for r in reqs:
        if r.status != "done":
            assert "cap" in r.error
            continue
        if r.key() not in solo:
            h, _ = backend.compile(r)
            try:
                solo[r.key()] = zx.sim_eval_amplitude(h)
            finally:
                zx.sim_program_free(h)
        assert r.result == solo[r.key()], r.rid
    fifo_reqs = S.make_stream(pool, 60, rate=400.0, seed=3)
    st2 = S.run_fifo(backend, fifo_reqs, realtime=True)
    for a, b in zip(reqs, fifo_reqs):
        assert a.status == b.status
        if a.status == "done":
            assert a.result == b.result


def test_autotuner_and_plan_agree_with_single_launches():
    from paper_2403_06777_amd import runtime
    qs = wl.batch_queries(48)
    hs = [zx.sim_compile(wl.circuit_text(c), zx.amplitude_query(y)) for c, y in qs]
    try:
        single = [zx.sim_eval_amplitude(h) for h in hs]
        best = runtime.autotune(hs, reps=1)
        plan = runtime.BatchPlan(hs, best)
        for _ in range(3):
            assert plan.run() == single
            assert zx.sim_eval_amplitude(hs[0]) == single[0]
        plan.free()
    finally:
        for h in hs:
            zx.sim_program_free(h)
