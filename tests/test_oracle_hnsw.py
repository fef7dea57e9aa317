"""Pins of the oracle's global HNSW construction (Alg. 7) and its layered search.

Layer draws are checked against hand-computed boundaries, against the
logarithm form floor(-ln U / ln M) and against the geometric law
P(l >= i) = M^-i.  The layers are checked structurally (nesting, complete
small layers by brute force, degree bounds, reachability from each layer's
entry point), and the layered search against brute force where it must be
exact (L >= n on a connected layer 0, greedy routing on complete layers).
"""
import math

import numpy as np
import pytest


def test_levels_hand_values(oracle):
    M = 4
    U = np.array([1.0, 0.5, 0.25, np.nextafter(0.25, 1.0), 1 / 16, np.nextafter(1 / 16, 1.0),
                  1 / 64, 1e-300])
    # 4^26 = 2^52 is the last power of 4 below 2^53: levels stop there
    assert list(oracle.hnsw_levels(U, M)) == [0, 0, 1, 0, 2, 1, 3, 26]


@pytest.mark.parametrize("M", [2, 5, 16, 32, 48])
def test_levels_match_logarithm_form_and_geometric_law(oracle, datagen, M):
    U = datagen.uniform_open01(200000, seed=M)
    lev = oracle.hnsw_levels(U, M)
    ref = np.floor(-np.log(U) / math.log(M)).astype(np.int64)
    # the two forms can differ only where -ln U / ln M rounds across an integer
    assert (lev != ref).sum() <= 2
    n = len(U)
    for i in range(1, 4):
        p = M ** -i
        got = (lev >= i).sum()
        assert abs(got - n * p) <= 5 * math.sqrt(n * p * (1 - p)) + 1, (i, got, n * p)


def _reach(ids, deg, start):
    seen = {start}
    stack = [start]
    while stack:
        v = stack.pop()
        for w in ids[v, :deg[v]].tolist():
            if w not in seen:
                seen.add(w)
                stack.append(w)
    return seen


@pytest.fixture(scope="module")
def hnsw(oracle, datagen):
    X, Q = datagen.sift_like(1500, 40, d=16, n_clusters=8, sigma=10.0, seed=23)
    U = datagen.uniform_open01(1500, seed=3)
    H = oracle.opt_hnsw(X, U, 12, 16, 6, 65.0, 1, 6, 6, 2, 0.001)
    return X, Q, U, H


def test_layers_nested_and_complete_layers_brute_force(oracle, hnsw):
    X, _, U, H = hnsw
    M = 6
    lev = oracle.hnsw_levels(U, M)
    assert H["max_level"] == lev.max() >= 2
    prev = None
    for i, lay in enumerate(H["layers"]):
        nodes = lay["nodes"]
        assert np.array_equal(nodes, np.nonzero(lev >= i)[0])
        if prev is not None:
            assert set(nodes.tolist()) <= set(prev.tolist())
        prev = nodes
        m = len(nodes)
        assert (lay["deg"] <= M).all()
        if m <= M:
            Xi = X[nodes].astype(np.float64)
            for u in range(m):
                others = [v for v in range(m) if v != u]
                want = sorted(others, key=lambda v: (((Xi[u] - Xi[v]) ** 2).sum(), v))
                assert list(lay["ids"][u, :m - 1]) == want
    assert H["ep"] in H["layers"][-1]["nodes"].tolist()


def test_large_layers_reachable_from_their_entry_point(oracle, hnsw):
    X, _, _, H = hnsw
    for lay in H["layers"]:
        m = len(lay["nodes"])
        if m <= 6:
            continue
        ep = oracle.entry_point(X[lay["nodes"]])
        assert len(_reach(lay["ids"], lay["deg"], ep)) == m


def test_layered_search_greedy_on_complete_top_layer_and_exact_at_full_width(oracle, hnsw):
    X, Q, _, H = hnsw
    n = len(X)
    # L = n on layer 0 (connected from every node after connect): brute force
    ids, d2 = oracle.hnsw_search(X, H, Q[:5], 10, n)
    gt, gd = oracle.exact_knn(X, Q[:5], 10)
    assert np.array_equal(ids, gt)
    # greedy routing on a complete layer reaches its exact nearest node
    top = H["layers"][H["max_level"]]
    assert len(top["nodes"]) <= 6
    Xt = X[top["nodes"]].astype(np.float64)
    for q in Q[:10].astype(np.float64):
        local = int(np.searchsorted(top["nodes"], H["ep"]))
        r, _, _ = oracle.search(X[top["nodes"]], top["ids"], top["deg"], q[None, :].astype(np.float32),
                                np.array([local], np.int32), 1, 1)
        dd = ((Xt - q) ** 2).sum(1)
        assert r[0, 0] == int(np.lexsort((np.arange(len(dd)), dd))[0])


def test_single_layer_equals_plain_search(oracle, datagen):
    X, Q = datagen.sift_like(800, 20, d=16, n_clusters=5, sigma=10.0, seed=4)
    U = np.ones(800)  # every node stays on layer 0
    H = oracle.opt_hnsw(X, U, 12, 16, 8, 62.0, 1, 6, 6, 5, 0.001)
    assert H["max_level"] == 0
    ids, _ = oracle.hnsw_search(X, H, Q, 10, 24)
    lay = H["layers"][0]
    for q in range(len(Q)):
        r, _, _ = oracle.search(X, lay["ids"], lay["deg"], Q[q:q + 1], np.array([H["ep"]], np.int32), 10, 24)
        assert np.array_equal(ids[q], r[0])
