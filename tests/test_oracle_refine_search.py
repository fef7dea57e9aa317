"""Pins of the oracle's refinement (Alg. 2 Phase 3) and beam search (Alg. 1).

Pins used: the PRUNE stage equals per-node Prune; the REVERSE stage output is
the Prune of the reverse union computed here independently; connectivity is
checked with an independent BFS; beam search with L >= n on a connected graph
and search on a complete graph return the brute-force answer.
"""
from collections import deque

import numpy as np
import pytest


def _reach(ids, deg, src):
    seen = {src}
    q = deque([src])
    while q:
        x = q.popleft()
        for y in ids[x, :deg[x]]:
            if y >= 0 and y not in seen:
                seen.add(int(y))
                q.append(int(y))
    return seen


def _knn_input(oracle, X, K):
    ids, _ = oracle.exact_knn(X, X, K, exclude=np.arange(len(X)))
    return ids


def test_prune_stage_is_per_node_prune(oracle, datagen):
    X = datagen.uniform_int(400, 12, seed=0)
    cand = _knn_input(oracle, X, 16)
    r = oracle.refine(X, cand, 8, stages=oracle.STAGE_PRUNE)
    for u in range(400):
        ref, rd = oracle.prune_one(X, u, cand[u], 8)
        assert list(r["ids"][u, :r["deg"][u]]) == list(ref)
        assert np.array_equal(r["d2"][u, :r["deg"][u]], rd)
        assert (r["ids"][u, r["deg"][u]:] == -1).all()


def test_reverse_stage(oracle, datagen):
    X = datagen.uniform_int(300, 10, seed=1)
    cand = _knn_input(oracle, X, 12)
    p = oracle.refine(X, cand, 6, stages=oracle.STAGE_PRUNE)
    r = oracle.refine(X, cand, 6, stages=oracle.STAGE_PRUNE | oracle.STAGE_REVERSE)
    rev = [[] for _ in range(300)]
    for v in range(300):
        for w in p["ids"][v, :p["deg"][v]]:
            rev[w].append(v)
    for u in range(300):
        union = list(p["ids"][u, :p["deg"][u]]) + rev[u]
        ref, _ = oracle.prune_one(X, u, union, 6)
        got = r["ids"][u, :r["deg"][u]]
        assert list(got) == list(ref)
        assert set(got.tolist()) <= set(int(x) for x in union)
        assert r["deg"][u] <= 6


def test_connect_reaches_everything(oracle, datagen):
    # well separated clusters: the pruned kNN graph is disconnected
    X, _ = datagen.sift_like(1200, 0, d=16, n_clusters=12, sigma=4.0, seed=5)
    cand = _knn_input(oracle, X, 10)
    no = oracle.refine(X, cand, 8, stages=oracle.STAGE_PRUNE | oracle.STAGE_REVERSE)
    before = _reach(no["ids"], no["deg"], no["ep"])
    assert len(before) < 1200
    r = oracle.refine(X, cand, 8)
    assert r["ep"] == oracle.entry_point(X)
    assert len(_reach(r["ids"], r["deg"], r["ep"])) == 1200
    assert (r["deg"] <= 8).all()
    # one extra edge per restart root; every root is a target of an added edge
    added = int((r["deg"] - no["deg"]).sum())
    assert added == len(r["roots"]) > 0
    assert r["roots"][0] == min(set(range(1200)) - before)
    for root in r["roots"]:
        assert (r["ids"] == root).any()


def test_search_large_pool_is_exact(oracle, datagen):
    X = datagen.uniform_int(500, 8, seed=2)
    Q = datagen.uniform_int(30, 8, seed=3)
    cand = _knn_input(oracle, X, 10)
    g = oracle.refine(X, cand, 8)
    assert len(_reach(g["ids"], g["deg"], g["ep"])) == 500
    ids, d2, st = oracle.search(X, g["ids"], g["deg"], Q, [g["ep"]], 10, 500)
    gt, gd = oracle.exact_knn(X, Q, 10)
    assert np.array_equal(ids, gt)
    assert np.array_equal(d2, gd)
    assert (st[:, 1] == 500).all()  # every node evaluated exactly once


def test_search_complete_graph_is_exact(oracle):
    rng = np.random.default_rng(8)
    n = 60
    X = rng.standard_normal((n, 5)).astype(np.float32)
    Q = rng.standard_normal((20, 5)).astype(np.float32)
    ids = np.array([[v for v in range(n) if v != u] for u in range(n)], np.int32)
    deg = np.full(n, n - 1, np.int32)
    got, gd, _ = oracle.search(X, ids, deg, Q, [0], 5, 5)
    gt, gtd = oracle.exact_knn(X, Q, 5)
    assert np.array_equal(got, gt)
    assert np.array_equal(gd, gtd)


def test_search_path_graph(oracle):
    # points 0..9 on a line, edges i -> i+1 only: from entry 0 with L = 1 the
    # beam walks to the end and returns the query's nearest reachable points
    X = np.arange(10, dtype=np.float32)[:, None]
    ids = np.array([[i + 1] if i < 9 else [-1] for i in range(10)], np.int32)
    deg = np.array([1] * 9 + [0], np.int32)
    got, d2, st = oracle.search(X, ids, deg, np.array([[6.2]], np.float32), [0], 1, 1)
    assert got[0, 0] == 6
    assert st[0, 0] == 7  # expands 0..6; 7 is evaluated but farther than 6


def test_multiple_entries_and_padding(oracle):
    X = np.arange(6, dtype=np.float32)[:, None]
    ids = np.full((6, 1), -1, np.int32)
    deg = np.zeros(6, np.int32)
    got, d2, _ = oracle.search(X, ids, deg, np.array([[4.4]], np.float32), [1, 4, 4, 0], 5, 8)
    assert list(got[0]) == [4, 1, 0, -1, -1]
    assert np.isinf(d2[0, 3:]).all()


def _py_connect(X, g_ids, g_deg, ep, cand, R):
    """Restatement of the connect reading: smallest unreached root r gets an
    edge from its closest reached candidate with spare degree (else the closest
    such reached node overall); then everything r reaches is marked."""
    ids, deg = g_ids.copy(), g_deg.copy()
    Xd = X.astype(np.float64)
    seen = _reach(ids, deg, ep)
    roots = []
    while len(seen) < len(X):
        r = min(set(range(len(X))) - seen)
        elig = [int(p) for p in cand[r] if p >= 0 and p != r and p in seen and deg[p] < R]
        if not elig:
            elig = [p for p in sorted(seen) if deg[p] < R]
        p = min(elig, key=lambda q: (float(((Xd[q] - Xd[r]) ** 2).sum()), q))
        ids[p, deg[p]] = r
        deg[p] += 1
        roots.append(r)
        seen |= _reach(ids, deg, r)
    return ids, deg, roots


def test_connect_matches_restatement(oracle, datagen):
    X, _ = datagen.sift_like(900, 0, d=8, n_clusters=9, sigma=3.0, seed=13)
    cand = _knn_input(oracle, X, 8)
    base = oracle.refine(X, cand, 6, stages=oracle.STAGE_PRUNE | oracle.STAGE_REVERSE)
    full = oracle.refine(X, cand, 6)
    ids, deg, roots = _py_connect(X, base["ids"], base["deg"], base["ep"], cand, 6)
    assert len(roots) > 0
    assert list(full["roots"]) == roots
    assert np.array_equal(full["deg"], deg)
    assert np.array_equal(full["ids"], ids)


# ------------------------------------------------ OptKCNA / IterNSG (Alg. 5, 6)

def test_search_self_complete_graph_is_exact_without_self(oracle):
    # complete graph: expanding the entry u evaluates every node, so the first
    # k pool entries other than u are the exact k nearest other points
    rng = np.random.default_rng(11)
    n = 80
    X = rng.standard_normal((n, 6)).astype(np.float32)
    ids = np.array([[v for v in range(n) if v != u] for u in range(n)], np.int32)
    deg = np.full(n, n - 1, np.int32)
    got, d2, _ = oracle.search_self(X, ids, deg, 7, 8)
    D = ((X[:, None, :].astype(np.float64) - X[None, :, :]) ** 2).sum(-1)
    for u in range(n):
        order = sorted((D[u, v], v) for v in range(n) if v != u)[:7]
        assert list(got[u]) == [v for _, v in order]
        assert np.allclose(d2[u], [dd for dd, _ in order], rtol=0, atol=1e-12)


def test_search_self_large_pool_is_exact(oracle, datagen):
    # L >= n on a connected graph: the search sees every node
    X = datagen.uniform_int(300, 8, seed=12)
    cand, _ = oracle.exact_knn(X, X, 10, exclude=np.arange(300))
    g = oracle.refine(X, cand, 8)
    got, d2, _ = oracle.search_self(X, g["ids"], g["deg"], 10, 300)
    assert np.array_equal(got, cand)
    assert (got != np.arange(300)[:, None]).all()


def test_opt_kcna_round_keeps_list_invariants(oracle, datagen):
    # one OptKCNA round on NN-Descent lists: lists stay sorted, self-free,
    # and (on integer data, where d2 is exact) their distances are the true ones
    X, _ = datagen.sift_like(1500, 0, d=16, n_clusters=10, sigma=6.0, seed=13)
    cand, _, _, _ = oracle.nndescent(X, 12, 6, 3, 1)
    ids, d2 = oracle.opt_kcna(X, cand, 12, 24, 8, 65.0)
    n = len(X)
    assert (ids != np.arange(n)[:, None]).all() and (ids >= 0).all()
    assert (np.diff(d2, axis=1) >= 0).all()
    true = ((X[np.arange(n)[:, None]].astype(np.float64) - X[ids]) ** 2).sum(-1)
    assert np.array_equal(true, d2)
    assert all(len(set(r)) == len(r) for r in ids.tolist())


def test_iter_nsg_zero_rounds_is_refined_nndescent(oracle, datagen):
    X, _ = datagen.sift_like(800, 0, d=16, n_clusters=8, sigma=6.0, seed=14)
    g = oracle.iter_nsg(X, 12, 6, 4, 3, 0, 12, 24, 8, 65.0, 0)
    cand, _, _, _ = oracle.nndescent(X, 12, 6, 4, 3, stop_updates=0)
    r = oracle.refine(X, cand, 8)
    assert np.array_equal(g["ids"], r["ids"]) and np.array_equal(g["cand"], cand)


# ------------------------------------------- quality examination (Section 5.2)

def test_quality_sample_size(oracle):
    # the theorem's bound, natural log: 1M points, eps = 0.6, l = 1 -> 354
    assert oracle.quality_sample_size(10**6, 0.6) == 354
    assert oracle.quality_sample_size(10**6, 0.6, l=2) == 707
    assert oracle.quality_sample_size(10**4, 0.3) > oracle.quality_sample_size(10**4, 0.6)


def test_quality_examination_known_lists(oracle, datagen):
    # exact lists score 1, lists of far points score 0, and lists whose first
    # half is exact score 1/2 exactly
    X = datagen.uniform_int(1500, 8, seed=21)
    n, k = len(X), 10
    exact, _ = oracle.exact_knn(X, X, 2 * k, exclude=np.arange(n))
    sample = datagen.sample_ids(n, 200, seed=3)
    assert oracle.quality_examination(X, exact, k, sample) == 1.0
    far = exact[:, k:2 * k]                 # ranks k..2k-1: none among the k nearest
    assert oracle.quality_examination(X, far, k, sample) == 0.0
    half = np.concatenate([exact[:, :k // 2], far[:, :k - k // 2]], axis=1)
    assert oracle.quality_examination(X, half, k, sample) == 0.5


def test_quality_estimate_concentrates(datagen):
    # the estimator on a sample of the theorem's size stays within eps/2 of
    # the true mean recall (per-node recalls drawn at random, many samples)
    import math
    rng = np.random.default_rng(4)
    n, eps = 5000, 0.2
    ns = int(math.ceil((8 + 2 * eps) * math.log(n) / eps ** 2))
    r = rng.integers(0, 11, size=n) / 10.0
    worst = max(abs(r[rng.choice(n, ns, replace=False)].mean() - r.mean()) for _ in range(300))
    assert worst < eps / 2


def test_iter_nsg_stops_on_quality(oracle, datagen):
    X, _ = datagen.sift_like(800, 0, d=16, n_clusters=8, sigma=6.0, seed=14)
    sample = datagen.sample_ids(len(X), 100, seed=5)
    g = oracle.iter_nsg(X, 12, 6, 4, 3, 0, 12, 24, 8, 65.0, 3, target=0.0, sample=sample)
    assert g["rounds"] == 0 and len(g["quality"]) == 1
    g = oracle.iter_nsg(X, 12, 6, 4, 3, 0, 12, 24, 8, 65.0, 2, target=1.01, sample=sample)
    assert g["rounds"] == 2 and len(g["quality"]) == 2
