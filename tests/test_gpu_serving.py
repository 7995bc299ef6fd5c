"""Continuous batching on the GPU: every request's result in the mix is identical to its
solo evaluation (tolerance 0), and equal to the one-launch-per-query baseline."""

import pytest

import paper_2403_06777_amd as zx
import paper_2403_06777_amd.serving as S
import workloads as wl

pytestmark = pytest.mark.gpu


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
