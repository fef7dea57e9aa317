"""FP64 replays of Alg. 3 (Prune, with the alpha test of Section 4.1) and
Alg. 1 (KANNSearch) that record how close each decision comes to its
threshold.  Test helper only: it explains differences between the GPU's FP32
results and the FP64 oracle's on float data, where the two sides see squared
distances that differ by rounding.

A squared distance evaluated as a chain of d fused multiply-adds in FP32 is
within (d + 2) u of the exact value, relatively (u = 2^-24, first order: one
rounding of each difference, doubled by squaring, and d accumulations of
nonnegative terms).  Two FP32 distances can therefore compare differently
from their exact values only when they lie within 2 (d + 2) u of each other
relative to their sum; the same scale bounds the change of the law-of-cosines
quantities a + b - c and 2 cos(alpha) sqrt(a b) relative to a + b + c.  A
decision whose normalised gap exceeds that band is taken identically by both
sides.
"""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24


def chain_band(d: int) -> float:
    """Relative band within which an FP32 chain decision may flip."""
    return 2.0 * (d + 2) * U32 * 1.01


def _gap(x: float, y: float) -> float:
    s = abs(x) + abs(y)
    return abs(x - y) / s if s > 0 else 0.0


def prune_replay(X, u, cand, R, alpha_deg=60.0, strict=False):
    """Alg. 3 in FP64 (the oracle's readings: u, -1 and repeats dropped, (d2, id)
    order).  Returns (kept ids, sorted candidate ids, per-candidate smallest
    normalised gap of the decisions that visiting it took, including its order
    against its neighbours in the sorted list)."""
    X64 = np.asarray(X, np.float64)
    ids = sorted({int(v) for v in cand if v >= 0 and v != u})
    d2u = {v: float(((X64[u] - X64[v]) ** 2).sum()) for v in ids}
    order = sorted(ids, key=lambda v: (d2u[v], v))
    gaps = np.full(len(order), np.inf)
    for j in range(len(order) - 1):
        g = _gap(d2u[order[j]], d2u[order[j + 1]])
        gaps[j] = min(gaps[j], g)
        gaps[j + 1] = min(gaps[j + 1], g)
    use_angle = alpha_deg > 60.0
    kappa = 0.0 if alpha_deg == 90.0 else 2.0 * math.cos(alpha_deg * math.pi / 180.0)
    kept = []
    for j, v in enumerate(order):
        if len(kept) >= R:
            break
        c = d2u[v]
        occluded = False
        for w in kept:
            a = d2u[w]
            b = float(((X64[v] - X64[w]) ** 2).sum())
            gaps[j] = min(gaps[j], _gap(b, c))
            if strict:
                gaps[j] = min(gaps[j], _gap(a, c))
            if not (b < c) or (strict and not (a < c)):
                continue
            if not use_angle or b == 0.0:
                occluded = True
                break
            t, r = a + b - c, kappa * math.sqrt(a * b)
            gaps[j] = min(gaps[j], abs(t - r) / (a + b + c))
            if t < r:
                occluded = True
                break
        if not occluded:
            kept.append(v)
    return kept, order, gaps


def prune_difference_explained(X, u, cand, R, gpu_row, alpha_deg=60.0, strict=False):
    """(explained, smallest gap, FP64 row).  A row that differs from the FP64
    replay is explained when some decision up to the first differing position
    lies within the band of the data's dimension."""
    ref, order, gaps = prune_replay(X, u, cand, R, alpha_deg, strict)
    gpu_row = [int(v) for v in gpu_row]
    if gpu_row == ref:
        return True, float(gaps.min()) if len(gaps) else math.inf, ref
    p = 0
    while p < min(len(ref), len(gpu_row)) and ref[p] == gpu_row[p]:
        p += 1
    pos = {v: i for i, v in enumerate(order)}
    last = len(order) - 1
    if p < len(ref) and p < len(gpu_row):
        last = max(pos.get(ref[p], last), pos.get(gpu_row[p], last))
    g = float(gaps[:last + 1].min()) if len(order) else math.inf
    return g <= chain_band(np.asarray(X).shape[1]), g, ref


def search_replay(X, g_ids, g_deg, q, entries, k, L):
    """Alg. 1 in FP64 exactly as the oracle runs it (entries, seen set, pool of
    L by (d2, id)).  Returns (first k ids, smallest normalised gap among the
    comparisons the search made: admission against the L-th key and the
    insertion position among pool neighbours)."""
    X64 = np.asarray(X, np.float64)
    q = np.asarray(q, np.float64)
    seen = set()
    pool = []  # [d2, id, expanded]
    ent = []
    for v in entries:
        v = int(v)
        if v < 0 or v >= len(X64) or v in seen:
            continue
        seen.add(v)
        ent.append(v)
    if ent:
        ev = ((X64[ent] - q) ** 2).sum(1)
        pool = sorted([[float(dv), v, False] for dv, v in zip(ev, ent)], key=lambda e: (e[0], e[1]))
    gmin = math.inf
    for j in range(min(len(pool), L + 1) - 1):
        gmin = min(gmin, _gap(pool[j][0], pool[j + 1][0]))
    pool = pool[:L]
    while True:
        i = next((i for i, e in enumerate(pool) if not e[2]), None)
        if i is None:
            break
        pool[i][2] = True
        x = pool[i][1]
        nb = [int(v) for v in g_ids[x][:g_deg[x]] if 0 <= v < len(X64) and int(v) not in seen]
        if not nb:
            continue
        dv = ((X64[nb] - q) ** 2).sum(1)
        for v, dd in zip(nb, dv.tolist()):
            seen.add(v)
            if len(pool) == L:
                gmin = min(gmin, _gap(dd, pool[-1][0]))
                if not ((dd, v) < (pool[-1][0], pool[-1][1])):
                    continue
            p = len(pool) if len(pool) < L else L - 1
            if len(pool) < L:
                pool.append(None)
            while p > 0 and (dd, v) < (pool[p - 1][0], pool[p - 1][1]):
                pool[p] = pool[p - 1]
                p -= 1
            pool[p] = [dd, v, False]
            if p > 0:
                gmin = min(gmin, _gap(dd, pool[p - 1][0]))
            if p + 1 < len(pool):
                gmin = min(gmin, _gap(dd, pool[p + 1][0]))
    return [e[1] for e in pool[:k]], gmin
