"""Scheduling logic of the continuous-batching server, driven on the CPU by a fake backend
whose partial sums identify exactly which slices were evaluated."""

import paper_2403_06777_amd.serving as S
from paper_2403_06777_amd import binding as B


class FakeBackend:
    """program of a request = n_slices slices; the raw partial of slices [f, f + c) is
    (sum of slice indices, count, 0, 0), so the finished sum shows every slice exactly once"""

    def __init__(self, image_bytes=1000, p_of=None, fail_on=None):
        self.image_bytes = image_bytes
        self.p_of = p_of or (lambda req: 10 + req.rid % 7)
        self.fail_on = fail_on or set()
        self.live = {}
        self.next = 1
        self.launches = []

    def compile(self, req):
        if req.rid in self.fail_on:
            raise B.SimError(B.SIM_ERANGE, "p exceeds the cap")
        p = self.p_of(req)
        h = self.next
        self.next += 1
        wb = min(p, 4)
        info = {"n_params": p, "walk_bits": wb, "n_slices": 1 << (p - wb), "is_zero": 0,
                "image_bytes": self.image_bytes}
        self.live[h] = info
        return h, info

    def eval_ranges(self, handles, firsts, counts):
        self.launches.append(len(handles))
        out = []
        for h, f, c in zip(handles, firsts, counts):
            assert h in self.live
            assert 0 <= f and f + c <= self.live[h]["n_slices"]
            out.append((sum(range(f, f + c)), c, 0, 0))
        return out

    def raw_add(self, a, b):
        return tuple(x + y for x, y in zip(a, b))

    def finalize(self, h, raw):
        return (raw, 0)

    def evaluate(self, h):
        n = self.live[h]["n_slices"]
        return ((n * (n - 1) // 2, n, 0, 0), 0)

    def free(self, h):
        assert h in self.live
        del self.live[h]


def _reqs(n, spacing=0.0):
    return [S.Request(i, i * spacing, f"circuit {i % 5}", "amplitude", bits=str(i % 3), n_qubits=1)
            for i in range(n)]


def test_every_request_gets_its_solo_result():
    be = FakeBackend()
    srv = S.Server(be, mem_budget=1 << 30, max_active=8, tick_terms=1 << 12, compile_workers=2)
    reqs = _reqs(40)
    st = srv.run(reqs, realtime=False)
    assert st.done == 40 and st.rejected == 0
    assert all(r.status == "done" for r in reqs)
    # results equal the solo value of the same program (each slice exactly once)
    for r in reqs:
        n = 1 << (r.p - min(r.p, 4))
        assert r.result == ((n * (n - 1) // 2, n, 0, 0), 0)
    assert max(be.launches) > 1  # launches were shared by several requests
    assert be.next - 1 <= 15     # repeated queries shared one compilation each
    srv.close()
    assert not be.live


def test_slot_limit_and_overlap():
    be = FakeBackend(p_of=lambda r: 16)
    srv = S.Server(be, mem_budget=1 << 30, max_active=3, tick_terms=1 << 10, compile_workers=1)
    st = srv.run(_reqs(10), realtime=False)
    assert st.done == 10
    assert max(be.launches) <= 3
    srv.close()


def test_memory_budget_holds_then_admits():
    be = FakeBackend(image_bytes=10_000)
    # room for two resident programs at a time (image + scratch per request)
    srv = S.Server(be, mem_budget=2 * (10_000 + 4096), max_active=8, tick_terms=1 << 10, compile_workers=4)
    reqs = [S.Request(i, 0.0, f"c{i}", "amplitude", bits="0", n_qubits=1) for i in range(6)]
    st = srv.run(reqs, realtime=False)
    assert st.done == 6 and st.rejected == 0
    assert st.held_for_memory > 0
    assert max(be.launches) <= 2
    srv.close()


def test_oversize_and_failing_programs_are_rejected_alone():
    be = FakeBackend(image_bytes=10_000, fail_on={3})
    srv = S.Server(be, mem_budget=5_000, max_active=8, tick_terms=1 << 10)
    reqs = _reqs(6)
    st = srv.run(reqs, realtime=False)
    assert st.rejected == 6  # every program is larger than the budget
    assert all(r.status == "rejected" for r in reqs)
    assert "EBUSY" in reqs[0].error and "cap" in reqs[3].error
    srv.close()
    be2 = FakeBackend(fail_on={2, 5})
    srv2 = S.Server(be2, mem_budget=1 << 30, max_active=4, tick_terms=1 << 10)
    reqs2 = [S.Request(i, 0.0, f"c{i}", "amplitude", bits="1", n_qubits=1) for i in range(8)]
    st2 = srv2.run(reqs2, realtime=False)
    assert st2.rejected == 2 and st2.done == 6
    assert reqs2[2].status == "rejected" and reqs2[0].status == "done"
    srv2.close()


def test_fifo_baseline_and_stats():
    be = FakeBackend()
    reqs = _reqs(12, spacing=0.001)
    st = S.run_fifo(be, reqs, realtime=True)
    assert st.done == 12
    summ = st.summary()
    assert summ["p50_s"] is not None and summ["p99_s"] >= summ["p50_s"]
    assert not be.live


def test_poisson_stream_mix():
    from workloads import serving_pool
    pool = serving_pool(4)
    reqs = S.make_stream(pool, 200, rate=100.0, seed=1)
    kinds = [r.kind for r in reqs]
    assert 0.15 < kinds.count("marginal") / len(kinds) < 0.45
    arr = [r.arrival for r in reqs]
    assert arr == sorted(arr) and 0.8 < arr[-1] / 2.0 < 1.25


class StepBackend(FakeBackend):
    """the one-step-per-tick interface: carried raw sums added and the last step finalised"""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.steps = []

    def step(self, handles, firsts, counts, carries, last):
        self.steps.append(list(zip(handles, counts, last)))
        out = []
        for h, f, c, carry, fin in zip(handles, firsts, counts, carries, last):
            assert h in self.live
            n = self.live[h]["n_slices"]
            assert 0 <= f and f + c <= n and fin == (f + c == n)
            raw = tuple(x + y for x, y in zip(carry, (sum(range(f, f + c)), c, 0, 0)))
            out.append((raw, 0) if fin else raw)
        return out


def test_step_interface_gives_solo_results():
    be = StepBackend()
    srv = S.Server(be, mem_budget=1 << 30, max_active=8, tick_terms=1 << 12, compile_workers=2)
    reqs = _reqs(40)
    st = srv.run(reqs, realtime=False)
    assert st.done == 40 and st.rejected == 0
    for r in reqs:
        n = 1 << (r.p - min(r.p, 4))
        assert r.result == ((n * (n - 1) // 2, n, 0, 0), 0)
    assert be.steps


def test_small_requests_overtake_a_large_one():
    # a large request (2^20 terms) is running when small ones (2^10) arrive: each small one
    # finishes in the tick after its admission, while the large one still progresses every tick
    sizes = {0: 20}
    be = StepBackend(p_of=lambda req: sizes.get(req.rid, 10))
    srv = S.Server(be, mem_budget=1 << 30, max_active=8, tick_terms=1 << 14, compile_workers=1,
                   alone_terms=1 << 14, lone_terms=1 << 14)
    reqs = _reqs(6)
    st = srv.run(reqs, realtime=False)
    assert st.done == 6
    big_ticks = [k for k, s in enumerate(be.steps) if any(h == 1 for h, _, _ in s)]
    for k, s in enumerate(be.steps):
        for h, c, fin in s:
            if h != 1:
                assert fin, (k, s)  # a small request's whole remainder fits the tick
            else:
                assert c > 0  # the large one moves in every tick it is active
    assert len(big_ticks) >= (1 << 20) // (1 << 14)


class PipeBackend(FakeBackend):
    """the pipelined interface: carried sums live in slots 'on the device', a step completes a
    few polls after it was enqueued, results are read per finished request"""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.carry = None
        self.tickets = []
        self.max_inflight = 0

    def open_pipeline(self, n_slots):
        self.carry = [None] * n_slots

    def enqueue_step(self, handles, firsts, counts, slots, flags):
        assert len(set(slots)) == len(slots)
        out = {}
        for k, (h, f, c, s, fl) in enumerate(zip(handles, firsts, counts, slots, flags)):
            n = self.live[h]["n_slices"]
            assert 0 <= f and f + c <= n and bool(fl & 2) == (f + c == n) and bool(fl & 1) == (f == 0)
            prev = (0, 0, 0, 0) if fl & 1 else self.carry[s]
            assert prev is not None
            raw = tuple(x + y for x, y in zip(prev, (sum(range(f, f + c)), c, 0, 0)))
            if fl & 2:
                out[k] = (raw, 0)
                self.carry[s] = None
            else:
                self.carry[s] = raw
        t = {"polls": 0, "out": out}
        self.tickets.append(t)
        live = sum(1 for x in self.tickets if x["polls"] < 2)
        self.max_inflight = max(self.max_inflight, live)
        return t

    def step_done(self, t):
        t["polls"] += 1
        return t["polls"] >= 2

    def step_wait(self, t):
        t["polls"] = 2

    def step_result(self, t, k):
        return t["out"][k]


def test_pipelined_loop_gives_solo_results():
    be = PipeBackend(p_of=lambda req: 9 + req.rid % 9)
    srv = S.Server(be, mem_budget=1 << 30, max_active=6, tick_terms=1 << 11, compile_workers=2)
    reqs = _reqs(60)
    st = srv.run(reqs, realtime=False, pipeline_depth=3)
    assert st.done == 60 and st.rejected == 0
    for r in reqs:
        n = 1 << (r.p - min(r.p, 4))
        assert r.result == ((n * (n - 1) // 2, n, 0, 0), 0), r.rid
    assert be.max_inflight >= 2  # steps overlapped
    assert all(x is None for x in be.carry)  # every slot released
