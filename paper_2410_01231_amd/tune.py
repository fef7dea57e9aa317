"""Autotuner of the build's result-invariant knobs.

The join path (the FP32 direct form, or exact MFMA tiles on integer data,
against 16-bit MFMA tiles with FP32 settling), the proposal bucket capacity
and the number of source passes of the first iteration change only the speed
of pg_knn_build, never its lists.  tune_knn() times the build for each
candidate setting on the caller's rows (after one untimed iteration that
allocates the setting's workspace, so the allocation is not timed) and keeps
the fastest.  By default it times the whole build the caller will run: a
prefix of the iterations can mislead, since the heaviest iterations come in
the middle and a bucket that overflows there forces a repeat pass (the
Deep-shaped set at the default capacity takes one in its third iteration).  The choice is cached per shape (rows rounded up to a
power of two, d, K, S and the join path the rows allow) in memory and, when
a path is given, in a JSON file, so later builds of the same shape skip the
probes.  knn_build_tuned() builds with the tuned knobs.
"""
from __future__ import annotations

import json
import os
import threading

from . import pg

_cache: dict[str, dict] = {}
_lock = threading.Lock()


def candidates(d: int, precision=None):
    """Knob settings tried for rows of dimension d: both join precisions (BF16
    for d <= 128 rows, FP16 otherwise: the 16-bit format the error bound
    favours at that width) or the given one, four bucket capacities and two
    pass counts.
    Larger buckets take fewer repeat passes after overflows on data whose
    hubs draw many proposals (the GIST-shaped set: 64 K slots per node cut
    its join from 1.42 to 1.29 s)."""
    half = pg.BF16 if d <= 128 else pg.FP16
    out = []
    for prec in ((pg.FP32, half) if precision is None else (precision,)):
        for B in (0, 16, 32, 64):     # 0: the default 8 K; else B x K
            for chunks in (0, 16):
                out.append({"precision": prec, "bucket_mult": B, "chunks": chunks})
    return out


def shape_key(n: int, d: int, K: int, S: int, join_path: str) -> str:
    p2 = 1
    while p2 < n:
        p2 *= 2
    return f"n{p2}-d{d}-K{K}-S{S}-{join_path}"


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, table):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(timings):
    """The fastest setting of [(ms, setting)] (ties: the earlier one)."""
    best = min(range(len(timings)), key=lambda i: (timings[i][0], i))
    ms, setting = timings[best]
    return dict(setting, ms=ms)


def _knobs(setting, K):
    B = setting["bucket_mult"] * K if setting["bucket_mult"] else 0
    return {"precision": setting["precision"], "bucket_cap": B, "chunks": setting["chunks"]}


def tune_knn(X, K, S=None, seed=0, max_iters=12, delta=0.001, probe_iters=None, cache_path=None, ctx=None,
             timer=None, precision=None):
    """Knobs for pg_knn_build on rows X: dict(precision, bucket_cap, chunks).
    The build timed is the one of (max_iters, delta), or with probe_iters the
    first probe_iters iterations without the stop rule.  timer(fn) -> ms runs
    fn and returns its duration (CUDA events by default).  precision, when
    given, fixes the join precision and tunes the other knobs for it (a cache
    entry of its own)."""
    import torch
    n, d = X.shape
    S = (K + 1) // 2 if S is None else S
    ctx = ctx or pg.context(X.device.index)
    # a first short build: warms the allocator and names the join path
    _, _, st = pg.knn_build(X, K, S=S, max_iters=1, seed=seed, ctx=ctx)
    key = shape_key(n, d, K, S, st["join_path"]) + ("" if precision is None else f"-p{precision}")
    with _lock:
        if key not in _cache:
            _cache.update(_load(cache_path))
        if key in _cache:
            return _knobs(_cache[key], K)

    def event_timer(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(ctx.stream)
        fn()
        b.record(ctx.stream)
        b.synchronize()
        return a.elapsed_time(b)
    timer = timer or event_timer
    # settings whose workspace would take more than half of the free memory are
    # skipped (memory the caching allocator holds counts as free)
    torch.cuda.empty_cache()
    free = torch.cuda.mem_get_info(X.device)[0]
    if probe_iters is None:
        run = dict(max_iters=max_iters, stop_updates=int(delta * n * K))
    else:
        run = dict(max_iters=probe_iters, stop_updates=-1)
    timings = []
    for setting in candidates(d, precision):
        kn = _knobs(setting, K)
        if setting["bucket_mult"] and pg.knn_workspace_bytes(n, d, K, S, precision=kn["precision"],
                                                            bucket_cap=kn["bucket_cap"]) > free // 2:
            continue
        pg.knn_build(X, K, S=S, max_iters=1, seed=seed, ctx=ctx, **kn)
        ms = timer(lambda: pg.knn_build(X, K, S=S, seed=seed, ctx=ctx, **run, **kn))
        timings.append((ms, setting))
    best = choose(timings)
    with _lock:
        _cache[key] = best
        if cache_path:
            table = _load(cache_path)
            table[key] = best
            _store(cache_path, table)
    return _knobs(best, K)


def lookup(n, d, K, S, join_path, precision=None, cache_path=None):
    """The cached knobs of a shape (join_path: that of the default FP32 build
    of the rows), or None when the shape has not been tuned."""
    key = shape_key(n, d, K, S, join_path) + ("" if precision is None else f"-p{precision}")
    with _lock:
        if key not in _cache:
            _cache.update(_load(cache_path))
        hit = _cache.get(key)
    return _knobs(hit, K) if hit is not None else None


def knn_build_tuned(X, K, S=None, max_iters=12, seed=0, delta=0.001, cache_path=None, ctx=None):
    """pg_knn_build with the tuned knobs of X's shape: (ids, d2, stats, knobs)."""
    kn = tune_knn(X, K, S=S, seed=seed, cache_path=cache_path, ctx=ctx)
    ids, d2, st = pg.knn_build(X, K, S=S, max_iters=max_iters, seed=seed, delta=delta, ctx=ctx, **kn)
    return ids, d2, st, kn
