"""Pins of the oracle's NN-Descent (initialization phase, Section 3.1; Exp. 12).

* K = n - 1 makes every list the exact neighbour list (brute force) after init.
* Every list holds K distinct ids other than its owner, sorted by (d2, id), and
  its stored d2 equals the recomputed value exactly.
* Element-wise monotonicity: the i-th d2 of a list never grows between
  iterations (the merge only admits closer candidates).
* A set-based pure-Python restatement of the same synchronous iteration,
  written independently from the C code, gives identical lists, flags and
  counters on tiny inputs.
* kNN recall against brute force on small clustered inputs is high.
"""
import numpy as np
import pytest

M64 = (1 << 64) - 1
GOLD = 0x9E3779B97F4A7C15


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _h(seed, stream, a, b):
    x = _mix((seed + GOLD * (stream + 1)) & M64)
    x = _mix((x + GOLD * (a + 1)) & M64)
    return _mix((x + GOLD * (b + 1)) & M64)


def _py_nndescent(X, K, S, T, seed):
    """Set-based restatement: state = {v: {id: (d2, is_new)}}."""
    Xd = X.astype(np.float64)
    n = len(X)

    def dist(a, b):
        return float(((Xd[a] - Xd[b]) ** 2).sum())

    lists = []
    for u in range(n):
        got, j = [], 0
        while len(got) < K:
            r = _h(seed, 0, u, j) % (n - 1)
            v = r + 1 if r >= u else r
            if v not in got:
                got.append(v)
            j += 1
        lists.append({v: (dist(u, v), True) for v in got})
    stats = []
    for t in range(1, T + 1):
        snap = [dict(L) for L in lists]
        nf, of = [], []
        for u in range(n):
            news = sorted((v for v, (_, f) in snap[u].items() if f),
                          key=lambda v: (_h(seed, 3 * t, u, v) >> 32, v))[:S]
            nf.append(set(news))
            of.append({v for v, (_, f) in snap[u].items() if not f})
            for v in news:
                snap[u][v] = (snap[u][v][0], False)
        rn = [[] for _ in range(n)]
        ro = [[] for _ in range(n)]
        for u in range(n):
            for v in nf[u]:
                rn[v].append(u)
            for v in of[u]:
                ro[v].append(u)
        new, old = [], []
        for u in range(n):
            a = set(sorted(rn[u], key=lambda w: (_h(seed, 3 * t + 1, u, w) >> 32, w))[:S])
            b = set(sorted(ro[u], key=lambda w: (_h(seed, 3 * t + 2, u, w) >> 32, w))[:S])
            new.append(nf[u] | a)
            old.append((of[u] | b) - new[u])
        kth = [max((d, v) for v, (d, _) in snap[v].items()) for v in range(n)]
        props = [set() for _ in range(n)]
        pairs = 0
        for u in range(n):
            nl, ol = sorted(new[u]), sorted(old[u])
            pairs += len(nl) * (len(nl) - 1) // 2 + len(nl) * len(ol)
            cand = [(a, b) for i, a in enumerate(nl) for b in nl[i + 1:]] + \
                   [(a, b) for a in nl for b in ol]
            for a, b in cand:
                dd = dist(a, b)
                if (dd, b) < kth[a]:
                    props[a].add((dd, b))
                if (dd, a) < kth[b]:
                    props[b].add((dd, a))
        updates = 0
        for v in range(n):
            merged = {w: (d, f, True) for w, (d, f) in snap[v].items()}
            for d, w in props[v]:
                if w not in merged:
                    merged[w] = (d, True, False)
            top = sorted(merged.items(), key=lambda kv: (kv[1][0], kv[0]))[:K]
            updates += sum(1 for _, (_, _, from_snap) in top if not from_snap)
            lists[v] = {w: (d, f) for w, (d, f, _) in top}
        stats.append((updates, pairs))
    ids = np.array([[w for w, _ in sorted(L.items(), key=lambda kv: (kv[1][0], kv[0]))]
                    for L in lists])
    flags = np.array([[int(L[w][1]) for w in row] for L, row in zip(lists, ids)])
    d2 = np.array([[L[w][0] for w in row] for L, row in zip(lists, ids)])
    return ids, d2, flags, stats


@pytest.mark.parametrize("seed,n,K,S,T", [(1, 30, 4, 2, 3), (2, 45, 6, 3, 4), (3, 25, 8, 8, 2)])
def test_matches_set_based_restatement(oracle, seed, n, K, S, T):
    rng = np.random.default_rng(seed)
    X = np.floor(rng.random((n, 4)) * 20).astype(np.float32)
    ids, d2, flags, st = oracle.nndescent(X, K, S, T, seed)
    rid, rd2, rfl, rst = _py_nndescent(X, K, S, T, seed)
    assert np.array_equal(ids, rid)
    assert np.array_equal(d2, rd2)
    assert np.array_equal(flags, rfl)
    assert [(u, p) for u, p in zip(st["updates"], st["pairs"])] == rst


def test_full_lists_are_exact(oracle):
    rng = np.random.default_rng(4)
    n = 40
    X = np.floor(rng.random((n, 5)) * 6).astype(np.float32)  # ties present
    gt, gd = oracle.exact_knn(X, X, n - 1, exclude=np.arange(n))
    for T in (0, 2):
        ids, d2, _, _ = oracle.nndescent(X, n - 1, 4, T, 7)
        assert np.array_equal(ids, gt)
        assert np.array_equal(d2, gd)


def test_list_invariants_and_monotonicity(oracle, datagen):
    X = datagen.uniform_int(600, 16, seed=0)
    prev = None
    Xd = X.astype(np.float64)
    for T in range(0, 5):
        ids, d2, flags, st = oracle.nndescent(X, 12, 6, T, 11)
        for u in range(0, 600, 7):
            row = ids[u]
            assert len(set(row.tolist())) == 12 and u not in row
            rd = ((Xd[row] - Xd[u]) ** 2).sum(1)
            assert np.array_equal(rd, d2[u])
            keys = list(zip(d2[u], row))
            assert keys == sorted(keys)
        if prev is not None:
            assert (d2 <= prev).all()
        prev = d2
        if T == 0:
            assert flags.all()


def test_updates_count_new_entries(oracle, datagen):
    X = datagen.uniform_int(300, 8, seed=3)
    a, _, _, _ = oracle.nndescent(X, 8, 4, 2, 5)
    b, _, fb, st = oracle.nndescent(X, 8, 4, 3, 5)
    changed = sum(len(set(b[v]) - set(a[v])) for v in range(300))
    assert st["updates"][2] == changed
    # every inserted entry is flagged new
    for v in range(300):
        for j, w in enumerate(b[v]):
            if w not in set(a[v]):
                assert fb[v, j] == 1


def test_recall_on_clusters(oracle, datagen):
    X, _ = datagen.sift_like(3000, 0, d=32, n_clusters=10, seed=2)
    ids, _, _, st = oracle.nndescent(X, 16, 8, 12, 3, stop_updates=int(0.001 * 3000 * 16))
    gt, _ = oracle.exact_knn(X, X, 16, exclude=np.arange(3000))
    rec = np.mean([len(set(a) & set(b)) / 16 for a, b in zip(ids, gt)])
    assert rec > 0.95, (rec, st)
