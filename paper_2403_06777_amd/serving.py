"""Continuous-batching server for amplitude and marginal queries.

Requests arrive over time (open loop).  Each is compiled on a host worker thread (the
reduction of Section 3 runs once per query), then admitted when a slot is free and its
program fits the device-memory budget; compiled programs stay resident in an LRU cache so
repeated queries skip compilation.  Every tick is ONE batched step on the device
(sim_serve_step): the next chunk of slices of every active request, each added to the raw
sum carried from its earlier ticks, and the requests whose last slices are in the tick
finalised in the same step and answered.  Requests that arrive while others are on the GPU
join the next tick: their work overlaps on the device with the requests already running.

Shares are size-aware: small requests take their whole remainder in the next tick (they do
not wait behind large ones), every request moves each tick, and the rest of the tick goes to
the large requests oldest first, in large chunks.  Up to `pipeline_depth` ticks are in flight on
the device, so the host prepares the next one while the device runs.

Because partial sums over disjoint slices add exactly in Z[w], a result does not depend
on how its slices were chunked or which other requests shared its launches: it is
bit-identical to a solo evaluation.

The backend is injectable (tests drive the scheduling logic with a fake one on the CPU);
ZxBackend is the real one over the C-ABI.
"""

import collections
import concurrent.futures as cf
import contextlib
import gc
import hashlib
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

from . import binding as B


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    circuit: str
    kind: str  # "amplitude" or "marginal"
    bits: str = ""
    n_qubits: int = 0
    qubit: int = 0
    value: int = 0
    status: str = "pending"  # done | rejected
    result: Optional[Tuple] = None
    error: str = ""
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    terms: int = 0
    p: int = -1

    def key(self) -> Tuple:
        h = hashlib.sha1(self.circuit.encode()).hexdigest()
        if self.kind == "amplitude":
            return (h, "a", self.bits)
        return (h, "m", self.n_qubits, self.qubit, self.value)

    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


class ZxBackend:
    """The library, through its C-ABI."""

    def __init__(self, stream=None, tuning: Optional[dict] = None, p_cap: int = 40):
        self.stream = stream
        self.tuning = tuning
        self.p_cap = p_cap

    def compile(self, req: Request):
        if req.kind == "amplitude":
            q = B.amplitude_query(req.bits)
        else:
            q = B.marginal_query(req.n_qubits, req.qubit, req.value)
        h = B.sim_compile(req.circuit, q, p_cap=self.p_cap)
        return h, B.sim_program_info(h)

    def eval_ranges(self, handles, firsts, counts):
        return B.sim_eval_ranges(handles, firsts, counts, self.stream, self.tuning)

    def step(self, handles, firsts, counts, carries, last):
        return B.sim_serve_step(handles, firsts, counts, carries, last, self.stream, self.tuning)

    # pipelined steps: carried sums in device slots, results copied back asynchronously
    def open_pipeline(self, n_slots: int):
        import torch
        self._torch = torch
        self._st = self.stream if self.stream is not None else torch.cuda.current_stream()
        self._n_slots = n_slots
        self._carry = torch.zeros(72 * n_slots + 256, dtype=torch.uint8, device="cuda")

    def enqueue_step(self, handles, firsts, counts, slots, flags):
        torch = self._torch
        n = len(handles)
        out = torch.empty(72 * n, dtype=torch.uint8, device="cuda")
        base = self._carry.data_ptr()
        base += (-base) % 8
        B.sim_serve_enqueue(handles, firsts, counts, slots, flags, base, self._n_slots, out.data_ptr(), self._st,
                            self.tuning)
        host = torch.empty(72 * n, dtype=torch.uint8, pin_memory=True)
        with torch.cuda.stream(self._st):
            host.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self._st)
        return (ev, host, out)

    def step_done(self, ticket) -> bool:
        return ticket[0].query()

    def step_wait(self, ticket):
        ticket[0].synchronize()

    def step_result(self, ticket, k: int):
        return B.zomega_from_bytes(ticket[1][72 * k:72 * (k + 1)].numpy().tobytes())

    def raw_add(self, a, b):
        return B.sim_raw_add(a, b)

    def finalize(self, handle, raw):
        return B.sim_finalize(handle, raw, self.stream)

    def finalize_many(self, handles, raws):
        return B.sim_finalize_batch(handles, raws, self.stream)

    def evaluate(self, handle):
        return B.sim_eval_amplitude(handle, self.stream)

    def free(self, handle):
        B.sim_program_free(handle)


@dataclass
class _Entry:
    handle: int
    info: dict
    bytes: int
    users: int = 0


@dataclass
class _Active:
    req: Request
    entry: _Entry
    next_slice: int = 0
    raw: Tuple = (0, 0, 0, 0)


@dataclass
class ServeStats:
    done: int = 0
    rejected: int = 0
    ticks: int = 0
    held_for_memory: int = 0
    cache_hits: int = 0
    terms: int = 0
    wall: float = 0.0
    latencies: List[float] = field(default_factory=list)

    def summary(self) -> dict:
        lat = sorted(self.latencies)

        def pct(q):
            if not lat:
                return None
            i = min(len(lat) - 1, max(0, int(round(q * (len(lat) - 1)))))
            return lat[i]

        return {"done": self.done, "rejected": self.rejected, "ticks": self.ticks,
                "held_for_memory": self.held_for_memory, "cache_hits": self.cache_hits,
                "terms": self.terms, "wall_s": self.wall,
                "terms_per_s": self.terms / self.wall if self.wall > 0 else None,
                "p50_s": pct(0.5), "p99_s": pct(0.99)}


class ProgramCache:
    """Resident compiled programs, LRU, bounded by a device-memory budget."""

    def __init__(self, backend, budget_bytes: int):
        self.backend = backend
        self.budget = budget_bytes
        self.entries: "collections.OrderedDict[Tuple, _Entry]" = collections.OrderedDict()
        self.used = 0

    def get(self, key) -> Optional[_Entry]:
        e = self.entries.get(key)
        if e is not None:
            self.entries.move_to_end(key)
        return e

    def make_room(self, need: int) -> bool:
        if need > self.budget:
            return False
        for key in list(self.entries.keys()):
            if self.used + need <= self.budget:
                break
            e = self.entries[key]
            if e.users == 0:
                self.backend.free(e.handle)
                self.used -= e.bytes
                del self.entries[key]
        return self.used + need <= self.budget

    def put(self, key, entry: _Entry):
        self.entries[key] = entry
        self.used += entry.bytes

    def clear(self):
        for e in self.entries.values():
            self.backend.free(e.handle)
        self.entries.clear()
        self.used = 0


@contextlib.contextmanager
def _collector_paused():
    """Pauses Python's cyclic garbage collector for the duration of a serving loop (both
    servers below): its full passes walk every object of the process and can stall a loop for
    tens of milliseconds, which shows up as tail latency.  The loops create no reference cycles
    that need it; it is restored (and runs as usual) afterwards."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


class Server:
    def __init__(self, backend, mem_budget: int = 64 << 20, max_active: int = 256, tick_terms: int = 1 << 28,
                 compile_workers: int = 4, scratch_per_request: int = 4096, alone_terms: int = 1 << 30,
                 small_terms: int = 1 << 24, lone_terms: int = 1 << 34):
        self.backend = backend
        self.cache = ProgramCache(backend, mem_budget)
        self.max_active = max_active
        self.tick_terms = tick_terms
        self.small_terms = small_terms
        # a request alone on the device takes up to alone_terms in one tick (the pipelined loop);
        # a lone request of at most lone_terms with nothing in flight is one blocking launch
        self.alone_terms = alone_terms
        self.lone_terms = lone_terms
        self.pool = cf.ThreadPoolExecutor(max_workers=compile_workers)
        self.scratch_per_request = scratch_per_request

    def close(self):
        self.pool.shutdown(wait=True)
        self.cache.clear()

    def _compile(self, req: Request):
        return self.backend.compile(req)

    def run(self, requests: List[Request], realtime: bool = True, pipeline_depth: int = 2) -> ServeStats:
        with _collector_paused():
            if pipeline_depth > 0 and hasattr(self.backend, "enqueue_step"):
                return self._run_pipelined(requests, realtime, pipeline_depth)
            return self._run_ticks(requests, realtime)

    def _run_ticks(self, requests: List[Request], realtime: bool) -> ServeStats:
        """The serving loop with one blocking device step per tick (backends without enqueue)."""
        stats = ServeStats()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        compiling: Dict[int, Tuple[Request, cf.Future]] = {}
        held: "collections.deque[Tuple[Request, int, dict]]" = collections.deque()  # compiled, no room yet
        waiting: "collections.deque[Tuple[Request, _Entry]]" = collections.deque()  # resident, pinned
        active: List[_Active] = []
        inflight: Dict[Tuple, cf.Future] = {}
        freed = set()  # handles of programs refused for size (shared by duplicate requests)
        start = time.perf_counter()
        now = lambda: time.perf_counter() - start  # noqa: E731

        def reject(req, msg):
            req.status, req.error, req.t_done = "rejected", msg, now()
            stats.rejected += 1

        def place(req, handle, info) -> bool:
            """make the compiled program resident (pinned) if the budget allows"""
            key = req.key()
            ent = self.cache.get(key)
            if ent is None:
                need = int(info["image_bytes"]) + self.scratch_per_request
                if need > self.cache.budget:
                    if handle not in freed:
                        self.backend.free(handle)
                        freed.add(handle)
                    inflight.pop(key, None)
                    reject(req, "SIM_EBUSY: program exceeds the device-memory budget")
                    return True
                if not self.cache.make_room(need):
                    return False
                ent = _Entry(handle, info, need)
                self.cache.put(key, ent)
            inflight.pop(key, None)
            ent.users += 1
            waiting.append((req, ent))
            return True

        while pending or compiling or held or waiting or active:
            t = now()
            # arrivals: resident programs are pinned and wait for a slot, others compile (in the
            # loop itself when nothing else is in flight: no hand-off to the pool)
            while pending and (pending[0].arrival <= t or not realtime):
                req = pending.popleft()
                key = req.key()
                ent = self.cache.get(key)
                if ent is not None:
                    stats.cache_hits += 1
                    ent.users += 1
                    waiting.append((req, ent))
                    continue
                fut = inflight.get(key)
                if fut is None:
                    idle = not (active or waiting or compiling or held)
                    if idle and not (pending and (pending[0].arrival <= t or not realtime)):
                        fut = cf.Future()
                        try:
                            fut.set_result(self._compile(req))
                        except B.SimError as e:
                            fut.set_exception(e)
                    else:
                        fut = self.pool.submit(self._compile, req)
                    inflight[key] = fut
                compiling[req.rid] = (req, fut)
            # finished compilations become resident when the memory budget allows
            for rid in list(compiling.keys()):
                req, fut = compiling[rid]
                if not fut.done():
                    continue
                del compiling[rid]
                try:
                    handle, info = fut.result()
                except B.SimError as e:
                    inflight.pop(req.key(), None)
                    reject(req, str(e))
                    continue
                if not place(req, handle, info):
                    stats.held_for_memory += 1
                    held.append((req, handle, info))
            for _ in range(len(held)):
                req, handle, info = held.popleft()
                if not place(req, handle, info):
                    held.append((req, handle, info))
            # admission to a slot
            while waiting and len(active) < self.max_active:
                req, ent = waiting.popleft()
                req.t_admit = now()
                req.p = ent.info["n_params"]
                req.terms = 1 << req.p
                if ent.info["is_zero"]:
                    req.result = self.backend.finalize(ent.handle, (0, 0, 0, 0))
                    self._finish(req, ent, stats, now())
                    continue
                active.append(_Active(req, ent))
            if not active:
                # idle: wake on the first finished compilation or the next arrival
                wait = 0.05
                if pending and realtime:
                    wait = min(wait, max(0.0, pending[0].arrival - now()))
                if compiling:
                    cf.wait([f for _, f in compiling.values()], timeout=wait, return_when=cf.FIRST_COMPLETED)
                elif held:
                    time.sleep(0.0002)
                elif pending and realtime and not waiting and wait > 0:
                    time.sleep(wait)
                continue
            if (len(active) == 1 and not waiting and not compiling and not held and active[0].next_slice == 0
                    and active[0].req.terms <= self.lone_terms):
                # a lone small request: one launch of its own, as fast as a dedicated queue
                a = active[0]
                a.req.result = self.backend.evaluate(a.entry.handle)
                stats.ticks += 1
                self._finish(a.req, a.entry, stats, now())
                active = []
                continue
            # one tick: the next chunk of every active request in one step on the device
            counts = self._shares(active)
            handles = [a.entry.handle for a in active]
            firsts = [a.next_slice for a in active]
            stats.ticks += 1
            still, finished = [], []
            if hasattr(self.backend, "step"):
                last = [a.next_slice + c >= a.entry.info["n_slices"] for a, c in zip(active, counts)]
                outs = self.backend.step(handles, firsts, counts, [a.raw for a in active], last)
                t_done = now()
                for a, cnt, out, fin in zip(active, counts, outs, last):
                    a.next_slice += cnt
                    if fin:
                        a.req.result = out
                        self._finish(a.req, a.entry, stats, t_done)
                    else:
                        a.raw = out
                        still.append(a)
                active = still
                continue
            raws = self.backend.eval_ranges(handles, firsts, counts)
            for a, cnt, raw in zip(active, counts, raws):
                a.raw = self.backend.raw_add(a.raw, raw)
                a.next_slice += cnt
                if a.next_slice >= a.entry.info["n_slices"]:
                    finished.append(a)
                else:
                    still.append(a)
            if finished:
                if hasattr(self.backend, "finalize_many"):
                    vals = self.backend.finalize_many([a.entry.handle for a in finished], [a.raw for a in finished])
                else:
                    vals = [self.backend.finalize(a.entry.handle, a.raw) for a in finished]
                t_done = now()
                for a, v in zip(finished, vals):
                    a.req.result = v
                    self._finish(a.req, a.entry, stats, t_done)
            active = still
        stats.wall = now()
        return stats

    def _shares(self, active: List[_Active]) -> List[int]:
        """Slices of each active request in the next tick.  Small requests (at most small_terms
        left) take their whole remainder, so they finish in the tick after their admission
        instead of waiting behind large ones; every other request moves by at least one slice;
        the rest of the tick's terms goes to the large requests in arrival order (oldest
        first), so they finish in about the order a FIFO queue would give them, with large
        chunks.  A request alone takes the larger alone_terms budget."""
        n = len(active)
        budget = self.alone_terms if n == 1 else self.tick_terms

        def per_slice(a):
            return max(1, (1 << a.entry.info["n_params"]) // a.entry.info["n_slices"])

        left = [a.entry.info["n_slices"] - a.next_slice for a in active]
        ps = [per_slice(a) for a in active]
        counts = [0] * n
        spent = 0
        for k in sorted(range(n), key=lambda k: left[k] * ps[k]):
            need = left[k] * ps[k]
            if need > self.small_terms or spent + need > budget:
                break
            counts[k] = left[k]
            spent += need
        for k in range(n):
            if counts[k] == 0 and left[k] > 0:
                counts[k] = 1
                spent += ps[k]
        for k in sorted(range(n), key=lambda k: active[k].req.arrival):
            room = budget - spent
            if room <= 0:
                break
            extra = min(left[k] - counts[k], room // ps[k])
            counts[k] += extra
            spent += extra * ps[k]
        return counts

    def _run_pipelined(self, requests: List[Request], realtime: bool, depth: int) -> ServeStats:
        """The serving loop with device-resident carried sums: up to `depth` steps are in flight
        on the device, and the next one is enqueued while they run, so the device never waits for
        the host between ticks; a request is answered when the step holding its last slices has
        completed (its result copied back asynchronously)."""
        stats = ServeStats()
        be = self.backend
        be.open_pipeline(self.max_active)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        compiling: Dict[int, Tuple[Request, cf.Future]] = {}
        held: "collections.deque[Tuple[Request, int, dict]]" = collections.deque()
        waiting: "collections.deque[Tuple[Request, _Entry]]" = collections.deque()
        active: List[_Active] = []
        inflight: "collections.deque[Tuple[object, List[Tuple[_Active, int]]]]" = collections.deque()
        free_slots = list(range(self.max_active - 1, -1, -1))
        slot_of: Dict[int, int] = {}
        inflight_keys: Dict[Tuple, cf.Future] = {}
        freed = set()
        start = time.perf_counter()
        now = lambda: time.perf_counter() - start  # noqa: E731

        def reject(req, msg):
            req.status, req.error, req.t_done = "rejected", msg, now()
            stats.rejected += 1

        def place(req, handle, info) -> bool:
            key = req.key()
            ent = self.cache.get(key)
            if ent is None:
                need = int(info["image_bytes"]) + self.scratch_per_request
                if need > self.cache.budget:
                    if handle not in freed:
                        be.free(handle)
                        freed.add(handle)
                    inflight_keys.pop(key, None)
                    reject(req, "SIM_EBUSY: program exceeds the device-memory budget")
                    return True
                if not self.cache.make_room(need):
                    return False
                ent = _Entry(handle, info, need)
                self.cache.put(key, ent)
            inflight_keys.pop(key, None)
            ent.users += 1
            waiting.append((req, ent))
            return True

        while pending or compiling or held or waiting or active or inflight:
            t = now()
            while pending and (pending[0].arrival <= t or not realtime):
                req = pending.popleft()
                key = req.key()
                ent = self.cache.get(key)
                if ent is not None:
                    stats.cache_hits += 1
                    ent.users += 1
                    waiting.append((req, ent))
                    continue
                fut = inflight_keys.get(key)
                if fut is None:
                    idle = not (active or waiting or compiling or held or inflight)
                    if idle and not (pending and (pending[0].arrival <= t or not realtime)):
                        fut = cf.Future()
                        try:
                            fut.set_result(self._compile(req))
                        except B.SimError as e:
                            fut.set_exception(e)
                    else:
                        fut = self.pool.submit(self._compile, req)
                    inflight_keys[key] = fut
                compiling[req.rid] = (req, fut)
            for rid in list(compiling.keys()):
                req, fut = compiling[rid]
                if not fut.done():
                    continue
                del compiling[rid]
                try:
                    handle, info = fut.result()
                except B.SimError as e:
                    inflight_keys.pop(req.key(), None)
                    reject(req, str(e))
                    continue
                if not place(req, handle, info):
                    stats.held_for_memory += 1
                    held.append((req, handle, info))
            for _ in range(len(held)):
                req, handle, info = held.popleft()
                if not place(req, handle, info):
                    held.append((req, handle, info))
            # completed steps: answer the requests whose last slices they held
            while inflight and be.step_done(inflight[0][0]):
                ticket, fin = inflight.popleft()
                t_done = now()
                for a, k in fin:
                    a.req.result = be.step_result(ticket, k)
                    free_slots.append(slot_of.pop(a.req.rid))
                    self._finish(a.req, a.entry, stats, t_done)
            # admission to a slot (each active request owns a carry slot until it is answered)
            while waiting and free_slots:
                req, ent = waiting.popleft()
                req.t_admit = now()
                req.p = ent.info["n_params"]
                req.terms = 1 << req.p
                if ent.info["is_zero"]:
                    req.result = be.finalize(ent.handle, (0, 0, 0, 0))
                    self._finish(req, ent, stats, now())
                    continue
                slot_of[req.rid] = free_slots.pop()
                active.append(_Active(req, ent))
            if (len(active) == 1 and not inflight and not waiting and not compiling and not held
                    and active[0].next_slice == 0 and active[0].req.terms <= self.lone_terms):
                # a lone small request: one launch of its own
                a = active[0]
                a.req.result = be.evaluate(a.entry.handle)
                stats.ticks += 1
                free_slots.append(slot_of.pop(a.req.rid))
                self._finish(a.req, a.entry, stats, now())
                active = []
                continue
            if active and len(inflight) < depth:
                counts = self._shares(active)
                handles = [a.entry.handle for a in active]
                firsts = [a.next_slice for a in active]
                slots = [slot_of[a.req.rid] for a in active]
                flags, fin, still = [], [], []
                for k, (a, c) in enumerate(zip(active, counts)):
                    last = a.next_slice + c >= a.entry.info["n_slices"]
                    flags.append((1 if a.next_slice == 0 else 0) | (2 if last else 0))
                    a.next_slice += c
                    (fin if last else still).append((a, k) if last else a)
                ticket = be.enqueue_step(handles, firsts, counts, slots, flags)
                stats.ticks += 1
                inflight.append((ticket, fin))
                active = still
                continue
            if inflight:
                # nothing else to enqueue: wait for the oldest step unless the host has work soon
                if not (compiling or (pending and realtime and pending[0].arrival - now() < 2e-4)):
                    be.step_wait(inflight[0][0])
                else:
                    time.sleep(0.00005)
                continue
            wait = 0.05
            if pending and realtime:
                wait = min(wait, max(0.0, pending[0].arrival - now()))
            if compiling:
                cf.wait([f for _, f in compiling.values()], timeout=wait, return_when=cf.FIRST_COMPLETED)
            elif held:
                time.sleep(0.0002)
            elif pending and realtime and not waiting and wait > 0:
                time.sleep(wait)
        stats.wall = now()
        return stats

    def _finish(self, req: Request, ent: _Entry, stats: ServeStats, t: float):
        ent.users -= 1
        req.status = "done"
        req.t_done = t
        stats.done += 1
        stats.terms += req.terms
        stats.latencies.append(req.latency())


def run_fifo(backend, requests: List[Request], realtime: bool = True, cache_budget: int = 64 << 20) -> ServeStats:
    """Baseline: one request at a time in arrival order, compiled (with the same resident
    program cache) and evaluated by one launch of its own."""
    with _collector_paused():
        return _run_fifo(backend, requests, realtime, cache_budget)


def _run_fifo(backend, requests: List[Request], realtime: bool, cache_budget: int) -> ServeStats:
    stats = ServeStats()
    cache = ProgramCache(backend, cache_budget)
    start = time.perf_counter()
    now = lambda: time.perf_counter() - start  # noqa: E731
    try:
        for req in sorted(requests, key=lambda r: r.arrival):
            if realtime:
                wait = req.arrival - now()
                if wait > 0:
                    time.sleep(wait)
            key = req.key()
            ent = cache.get(key)
            if ent is None:
                try:
                    handle, info = backend.compile(req)
                except B.SimError as e:
                    req.status, req.error, req.t_done = "rejected", str(e), now()
                    stats.rejected += 1
                    continue
                ent = _Entry(handle, info, int(info["image_bytes"]))
                cache.make_room(ent.bytes)
                cache.put(key, ent)
            else:
                stats.cache_hits += 1
            req.t_admit = now()
            req.p = ent.info["n_params"]
            req.terms = 1 << req.p
            req.result = backend.evaluate(ent.handle)
            req.status = "done"
            req.t_done = now()
            stats.done += 1
            stats.terms += req.terms
            stats.latencies.append(req.latency())
    finally:
        stats.wall = now()
        cache.clear()
    return stats


def make_stream(pool, n_requests: int, rate: float, seed: int = 0, marginal_frac: float = 0.3) -> List[Request]:
    """Poisson arrivals at `rate` per second; each request picks a pool circuit, and is a
    marginal P(q = v) with probability marginal_frac, else an amplitude of a random string."""
    import math
    from workloads import SplitMix64, circuit_text

    rng = SplitMix64(40, seed)
    t = 0.0
    out = []
    texts = [circuit_text(c) for c in pool]
    for i in range(n_requests):
        t += -math.log(1.0 - rng.uniform()) / rate
        ci = rng.randint(0, len(pool) - 1)
        c = pool[ci]
        if rng.uniform() < marginal_frac:
            out.append(Request(i, t, texts[ci], "marginal", n_qubits=c.n_qubits,
                               qubit=rng.randint(0, c.n_qubits - 1), value=rng.randint(0, 1)))
        else:
            bits = "".join("1" if rng.bernoulli(0.5) else "0" for _ in range(c.n_qubits))
            out.append(Request(i, t, texts[ci], "amplitude", bits=bits, n_qubits=c.n_qubits))
    return out
