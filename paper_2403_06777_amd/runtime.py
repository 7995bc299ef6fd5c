"""Batch runtime: autotuned launch shapes and replayable batch plans.

A batch of compiled programs is cut into work items of about 2^chunk_log2 terms (slice ranges
of one program); each kernel variant takes its items in one launch, one workgroup per item, and
programs of 2^26 terms or more get resident-grid launches of their own.  The launch sequence is
captured once into a hipGraph by the library (sim_batch_plan_create) and replayed.  The autotuner times a few launch shapes (threads per workgroup, resident
workgroups per CU, terms per work item) on the actual batch and caches the winner under a
key that summarises the batch (parameter-count histogram and form widths).
"""

import json
import os
import time
from typing import Dict, List, Optional, Sequence

from . import binding as B

DEFAULT_CANDIDATES = [
    {"block_threads": 256, "chunk_log2": 20},
    {"block_threads": 256, "chunk_log2": 22},
    {"block_threads": 256, "chunk_log2": 24},
    {"block_threads": 128, "chunk_log2": 20},
    {"block_threads": 128, "chunk_log2": 22},
    {"block_threads": 256, "chunk_log2": 18},
]

_CACHE: Dict[str, dict] = {}
CACHE_PATH = os.environ.get("ZXPAR_TUNE_CACHE", "")


def batch_key(handles: Sequence[int]) -> str:
    hist = {}
    widths = set()
    for h in handles:
        info = B.sim_program_info(h)
        bucket = min(64, info["n_params"] // 4 * 4)
        hist[bucket] = hist.get(bucket, 0) + 1
        widths.add(max(1, (info["n_forms"] + 31) // 32))
    return json.dumps({"p": sorted(hist.items()), "w": sorted(widths)})


def _load_cache():
    if CACHE_PATH and os.path.exists(CACHE_PATH) and not _CACHE:
        with open(CACHE_PATH) as f:
            _CACHE.update(json.load(f))


def _save_cache():
    if CACHE_PATH:
        with open(CACHE_PATH, "w") as f:
            json.dump(_CACHE, f)


def time_plan(handles: Sequence[int], tuning: Optional[dict], reps: int = 2, stream=None):
    """wall seconds of one replay of a captured batch plan (best of reps, after a warm run)"""
    plan = B.sim_batch_plan_create(list(handles), tuning, stream)
    try:
        res = B.sim_batch_plan_run(plan, len(handles), stream)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            B.sim_batch_plan_run(plan, len(handles), stream)
            best = min(best, time.perf_counter() - t0)
        return best, res
    finally:
        B.sim_batch_plan_free(plan)


def autotune(handles: Sequence[int], candidates: Optional[List[dict]] = None, reps: int = 2,
             stream=None) -> dict:
    """Best launch shape for this batch; results of every candidate must agree exactly."""
    _load_cache()
    key = batch_key(handles)
    if key in _CACHE:
        return dict(_CACHE[key])
    best, best_t, ref = None, float("inf"), None
    for cand in candidates or DEFAULT_CANDIDATES:
        t, res = time_plan(handles, cand, reps, stream)
        if ref is None:
            ref = res
        elif res != ref:
            raise RuntimeError(f"launch shape {cand} changed a result")
        if t < best_t:
            best, best_t = cand, t
    _CACHE[key] = dict(best)
    _save_cache()
    return dict(best)


class BatchPlan:
    """A captured, replayable evaluation of a fixed batch of programs."""

    def __init__(self, handles: Sequence[int], tuning: Optional[dict] = None, stream=None):
        self.handles = list(handles)
        self.tuning = tuning
        self.plan = B.sim_batch_plan_create(self.handles, tuning, stream)

    def run(self, stream=None):
        return B.sim_batch_plan_run(self.plan, len(self.handles), stream)

    def free(self):
        if self.plan:
            B.sim_batch_plan_free(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
