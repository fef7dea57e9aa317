"""The FP64 replays in tests/neartie.py (used to explain float-data
differences between the GPU and the oracle) reproduce the oracle's Alg. 3
and Alg. 1 exactly, and their decision gaps behave as stated."""
import numpy as np
import pytest

import neartie


@pytest.mark.parametrize("alpha", [60.0, 65.0, 90.0, 120.0])
def test_prune_replay_equals_oracle(oracle, datagen, alpha):
    X, _ = datagen.gist_like(300, 0, d=24, n_clusters=4, seed=41)
    cand, _ = oracle.exact_knn(X, X, 20, exclude=np.arange(300, dtype=np.int32))
    for u in range(0, 300, 7):
        ref, _ = oracle.prune_one(X, u, cand[u], 8, alpha_deg=alpha)
        kept, order, gaps = neartie.prune_replay(X, u, cand[u], 8, alpha_deg=alpha)
        assert kept == list(ref)
        assert len(gaps) == len(order) and (gaps >= 0).all()
        ok, g, rep = neartie.prune_difference_explained(X, u, cand[u], 8, list(ref), alpha_deg=alpha)
        assert ok and rep == kept


def test_prune_difference_explained_only_near_ties(oracle):
    # u at the origin; nodes at squared distances 1, 4, 9 and 9 (1 + 2^-23):
    # swapping the last two (a difference an FP32 rounding could cause) is
    # explained, swapping the first two is not
    X = np.array([[0, 0, 0, 0], [1, 0, 0, 0], [0, 2, 0, 0], [0, 0, 3, 0],
                  [0, 0, 0, np.nextafter(np.float32(3), np.float32(4))]], np.float32)
    cand = np.array([1, 2, 3, 4], np.int32)
    kept, order, gaps = neartie.prune_replay(X, 0, cand, 4)
    assert kept == [1, 2, 3, 4]
    ref, _ = oracle.prune_one(X, 0, cand, 4)
    assert kept == list(ref)
    ok, g, _ = neartie.prune_difference_explained(X, 0, cand, 4, [1, 2, 4, 3])
    assert ok and g < neartie.chain_band(4)
    ok, g, _ = neartie.prune_difference_explained(X, 0, cand, 4, [2, 1, 3, 4])
    assert not ok and g > 0.1


def test_search_replay_equals_oracle(oracle, datagen):
    X, Q = datagen.gist_like(1500, 20, d=32, n_clusters=5, seed=42)
    cand, _ = oracle.exact_knn(X, X, 16, exclude=np.arange(1500, dtype=np.int32))
    r = oracle.refine(X, cand, 10)
    entries = np.concatenate([[r["ep"]], datagen.sample_ids(1500, 15, seed=3)]).astype(np.int32)
    rid, _, _ = oracle.search(X, r["ids"], r["deg"], Q, entries, 10, 40)
    for i in range(len(Q)):
        ids, gmin = neartie.search_replay(X, r["ids"], r["deg"], Q[i], entries, 10, 40)
        assert ids == list(rid[i])
        assert gmin >= 0.0
