"""Pins of the oracle's generator, brute-force kNN, entry point and recall.

Each test checks the oracle against something other than itself: published
generator outputs, a numpy full-matrix brute force, closed forms on points on
a line, or a hand-counted recall.
"""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


def _golden_splitmix():
    rows = []
    with open(os.path.join(HERE, "golden", "splitmix64_state0.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                i, h = line.split()
                rows.append((int(i), int(h, 16)))
    return rows


def test_splitmix_published_outputs(oracle):
    for i, h in _golden_splitmix():
        assert oracle.splitmix(0, i) == h


def test_hash_is_nested_splitmix(oracle):
    # h(seed, stream, a, b) = sm(sm(sm(seed, stream+1), a+1), b+1)
    for seed, stream, a, b in [(0, 0, 0, 0), (7, 3, 11, 5), (2**63 + 5, 40, 999999, 123456)]:
        x = oracle.splitmix(seed, stream + 1)
        x = oracle.splitmix(x, a + 1)
        assert oracle.hash64(seed, stream, a, b) == oracle.splitmix(x, b + 1)


def test_hash_uniform_mod(oracle):
    # 16 buckets of 20,000 draws: chi-square with 15 dof stays far below 50
    cnt = np.zeros(16)
    for j in range(20000):
        cnt[oracle.hash64(1, 0, 17, j) % 16] += 1
    chi2 = float(((cnt - 1250.0) ** 2 / 1250.0).sum())
    assert chi2 < 50.0


def _numpy_knn(X, Q, k, exclude=None):
    X = X.astype(np.float64)
    Q = Q.astype(np.float64)
    D = ((Q[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    ids = np.empty((len(Q), k), np.int64)
    d2 = np.empty((len(Q), k))
    for q in range(len(Q)):
        order = np.lexsort((np.arange(len(X)), D[q]))
        if exclude is not None:
            order = order[order != exclude[q]]
        ids[q] = order[:k]
        d2[q] = D[q, order[:k]]
    return ids, d2


@pytest.mark.parametrize("d", [1, 3, 17])
def test_exact_knn_matches_full_matrix(oracle, d):
    rng = np.random.default_rng(d)
    X = np.floor(rng.random((300, d)) * 8).astype(np.float32)  # many ties
    Q = np.floor(rng.random((40, d)) * 8).astype(np.float32)
    ids, d2 = oracle.exact_knn(X, Q, 12)
    rid, rd2 = _numpy_knn(X, Q, 12)
    assert np.array_equal(ids, rid)
    assert np.array_equal(d2, rd2)
    # data as queries: self excluded
    ids, d2 = oracle.exact_knn(X, X[:50], 7, exclude=np.arange(50))
    rid, rd2 = _numpy_knn(X, X[:50], 7, exclude=np.arange(50))
    assert np.array_equal(ids, rid)
    assert np.array_equal(d2, rd2)


def test_exact_knn_points_on_line(oracle):
    # x_i = i on a line: the k nearest of point i are i-1, i+1, i-2, i+2, ...
    # with the smaller id first at equal distance; d2 = 1, 1, 4, 4, ...
    n = 50
    X = np.arange(n, dtype=np.float32)[:, None]
    ids, d2 = oracle.exact_knn(X, X, 4, exclude=np.arange(n))
    for i in range(2, n - 2):
        assert list(ids[i]) == [i - 1, i + 1, i - 2, i + 2]
        assert list(d2[i]) == [1.0, 1.0, 4.0, 4.0]
    # fewer than k points: padded
    ids, d2 = oracle.exact_knn(X[:3], X[:1], 5, exclude=np.array([0]))
    assert list(ids[0]) == [1, 2, -1, -1, -1]
    assert np.isinf(d2[0, 2:]).all()


def test_entry_point_is_closest_to_centroid(oracle):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((777, 9)).astype(np.float32)
    c = X.astype(np.float64).mean(0)
    dd = ((X.astype(np.float64) - c) ** 2).sum(1)
    assert oracle.entry_point(X) == int(np.argmin(dd))
    # symmetric configuration: the centroid is the origin, two points tie; smaller id wins
    Y = np.array([[3, 0], [1, 0], [-1, 0], [-3, 0]], np.float32)
    assert oracle.entry_point(Y) == 1


def test_recall_hand_count(oracle):
    found = np.array([[1, 2, 3], [4, 5, -1]])
    true = np.array([[3, 2, 9], [7, 8, 9]])
    assert oracle.recall_at_k(found, true) == pytest.approx(2 / 6)
