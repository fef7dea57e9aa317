"""Pins of the oracle's Prune (Alg. 3, alpha test of Section 4.1) and refinement.

Pins used: hand-checked integer cases (tests/golden/prune_cases.json), a
brute-force enumeration showing the greedy output is the unique set with the
occlusion and maximality properties, angles measured with arccos instead of the
law of cosines, the alpha = 60 degree equivalence with RNG pruning, and
closed forms (alpha >= 180 keeps the first M).
"""
import itertools
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _cases():
    with open(os.path.join(HERE, "golden", "prune_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_cases(oracle, case):
    X = np.array(case["points"], np.float32)
    ids, _ = oracle.prune_one(X, case["u"], case["cand"], case["R"], alpha_deg=case["alpha"],
                              strict_ties=case["strict"])
    assert list(ids) == case["expect"], case["why"]


def _angle_deg(pu, pw, pv):
    a = pu - pw
    b = pv - pw
    cosv = float(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))
    return float(np.degrees(np.arccos(np.clip(cosv, -1.0, 1.0))))


def _occludes(X, u, w, v, alpha, strict):
    """Does kept w occlude v for node u (distances in float64, angle via arccos)?"""
    Xd = X.astype(np.float64)
    a = ((Xd[u] - Xd[w]) ** 2).sum()
    b = ((Xd[v] - Xd[w]) ** 2).sum()
    c = ((Xd[u] - Xd[v]) ** 2).sum()
    if not b < c:
        return False
    if strict and not a < c:
        return False
    if alpha <= 60:
        return True
    if b == 0:
        return True
    return _angle_deg(Xd[u], Xd[w], Xd[v]) > alpha


def _order(X, u, cand):
    Xd = X.astype(np.float64)
    ids = sorted({int(c) for c in cand if c >= 0 and c != u})
    return sorted(ids, key=lambda v: (((Xd[u] - Xd[v]) ** 2).sum(), v))


def _valid(X, u, order, S, R, alpha, strict):
    """Occlusion invariant + maximality up to the point where |S| reaches R."""
    kept = []
    for v in order:
        if len(kept) == R:
            if v in S:
                return False
            continue
        occl = any(_occludes(X, u, w, v, alpha, strict) for w in kept)
        if (v in S) == occl:
            return False
        if v in S:
            kept.append(v)
    return set(kept) == set(S)


@pytest.mark.parametrize("seed", range(6))
def test_greedy_is_unique_valid_subset(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    X = np.floor(rng.random((12, 3)) * 10).astype(np.float32)
    u = 0
    cand = rng.integers(0, 12, size=10)
    R = int(rng.integers(1, 6))
    order = _order(X, u, cand)
    for alpha, strict in [(60, False), (60, True), (75, False), (110, False)]:
        valid = []
        for r in range(0, min(R, len(order)) + 1):
            for S in itertools.combinations(order, r):
                if _valid(X, u, order, set(S), R, alpha, strict):
                    valid.append(set(S))
        assert len(valid) == 1
        ids, _ = oracle.prune_one(X, u, cand, R, alpha_deg=alpha, strict_ties=strict)
        assert set(ids.tolist()) == valid[0]
        # output is in visiting order
        assert list(ids) == [v for v in order if v in valid[0]]


@pytest.mark.parametrize("seed", range(4))
def test_alpha60_equals_rng(oracle, seed):
    # the angle test evaluated at exactly 60 degrees never changes the outcome
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((400, 8)).astype(np.float32)
    for u in range(0, 400, 37):
        cand = rng.choice(400, size=64, replace=False)
        a, _ = oracle.prune_one(X, u, cand, 16, alpha_deg=60.0)
        b, _ = oracle.prune_one(X, u, cand, 16, alpha_deg=60.0, force_angle=True)
        assert np.array_equal(a, b)


def test_alpha_larger_keeps_superset_order_prefix(oracle):
    # alpha >= 180: no angle exceeds it, nothing is occluded; the first M are kept
    rng = np.random.default_rng(3)
    X = rng.standard_normal((200, 5)).astype(np.float32)
    cand = rng.choice(200, size=40, replace=False)
    ids, _ = oracle.prune_one(X, 7, cand, 12, alpha_deg=180.0)
    assert list(ids) == _order(X, 7, cand)[:12]


@pytest.mark.parametrize("alpha", [60.0, 67.0, 100.0])
def test_random_float_characterisation(oracle, alpha):
    rng = np.random.default_rng(int(alpha))
    X = rng.standard_normal((300, 16)).astype(np.float32)
    for u in range(0, 300, 29):
        cand = rng.choice(300, size=48, replace=False)
        ids, d2 = oracle.prune_one(X, u, cand, 10, alpha_deg=alpha)
        order = _order(X, u, cand)
        assert _valid(X, u, order, set(ids.tolist()), 10, alpha, False)
        assert ids[0] == order[0]  # the nearest candidate is always kept
        assert len(ids) <= 10


def test_prune_table_matches_data_path(oracle):
    # integer data: float32 tables of squared distances are exact
    rng = np.random.default_rng(9)
    n, C, R = 60, 12, 5
    X = np.floor(rng.random((n, 6)) * 50).astype(np.float32)
    cand = np.stack([rng.choice(np.delete(np.arange(n), u), size=C, replace=False)
                     for u in range(n)]).astype(np.int32)
    pos = np.concatenate([np.arange(n)[:, None], cand], 1)
    P = X.astype(np.float64)[pos]
    tab = ((P[:, :, None, :] - P[:, None, :, :]) ** 2).sum(-1).astype(np.float32)
    ids, d2, deg = oracle.prune_table(cand, tab, R)
    for u in range(n):
        ref, _ = oracle.prune_one(X, u, cand[u], R)
        assert list(ids[u, :deg[u]]) == list(ref)
        assert (ids[u, deg[u]:] == -1).all()
