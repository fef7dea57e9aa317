"""ctypes binding of the FP64 CPU oracle (``pg_oracle.c``).

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg import this module.  The product library never does, and this
module imports nothing from the product package.  Every function returns numpy
arrays; distances are float64 squared L2 distances.  See the header of
``pg_oracle.c`` for the passage of the paper each function follows and the
readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

STAGE_PRUNE, STAGE_REVERSE, STAGE_CONNECT = 1, 2, 4
STAGES_ALL = STAGE_PRUNE | STAGE_REVERSE | STAGE_CONNECT


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE double: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u32, u64, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                               ctypes.c_uint64, ctypes.c_double)
    lib.orc_splitmix.restype = u64
    lib.orc_splitmix.argtypes = [u64, u64]
    lib.orc_hash.restype = u64
    lib.orc_hash.argtypes = [u64, u64, u64, u64]
    lib.orc_exact_knn.restype = ctypes.c_int
    lib.orc_exact_knn.argtypes = [P, i64, i32, i64, P, i64, i64, P, i32, P, P]
    lib.orc_nndescent.restype = ctypes.c_int
    lib.orc_nndescent.argtypes = [P, i64, i32, i64, i32, i32, i32, i64, u64, P, P, P, P]
    lib.orc_prune_one.restype = i32
    lib.orc_prune_one.argtypes = [P, i64, i32, i32, P, i32, i32, f64, i32, i32, P, P]
    lib.orc_prune_table.restype = ctypes.c_int
    lib.orc_prune_table.argtypes = [i64, P, i32, P, i32, f64, i32, P, P, P]
    lib.orc_entry_point.restype = i32
    lib.orc_entry_point.argtypes = [P, i64, i32, i64]
    lib.orc_refine.restype = ctypes.c_int
    lib.orc_refine.argtypes = [P, i64, i32, i64, P, i32, i32, f64, i32, u32, P, P, P, P, P, P]
    lib.orc_search.restype = ctypes.c_int
    lib.orc_search.argtypes = [P, i64, i32, i64, P, i32, P, P, i64, i64, P, i32, i32, i32,
                               P, P, P]
    lib.orc_search_self.restype = ctypes.c_int
    lib.orc_search_self.argtypes = [P, i64, i32, i64, P, i32, P, i32, i32, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(X):
    return np.ascontiguousarray(X, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def splitmix(state: int, i: int) -> int:
    """i-th output (i >= 1) of SplitMix64 started at the given state."""
    return int(_load().orc_splitmix(state, i))


def hash64(seed: int, stream: int, a: int, b: int) -> int:
    return int(_load().orc_hash(seed, stream, a, b))


def exact_knn(X, Q, k, exclude=None):
    """Brute-force k nearest neighbours of each row of Q among the rows of X."""
    lib = _load()
    X, Q = _f32(X), _f32(Q)
    n, d = X.shape
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.int32)
    d2 = np.empty((nq, k), np.float64)
    ex = None if exclude is None else _i32(exclude)
    _check(lib.orc_exact_knn(_ptr(X), n, d, d, _ptr(Q), nq, d,
                             None if ex is None else _ptr(ex), k, _ptr(ids), _ptr(d2)),
           "exact_knn")
    return ids, d2


def nndescent(X, K, S, max_iters, seed, stop_updates=-1):
    """Deterministic synchronous NN-Descent; returns ids, d2, flags, stats dict."""
    lib = _load()
    X = _f32(X)
    n, d = X.shape
    ids = np.empty((n, K), np.int32)
    d2 = np.empty((n, K), np.float64)
    flags = np.empty((n, K), np.uint8)
    stats = np.zeros(1 + 2 * max(max_iters, 0), np.int64)
    _check(lib.orc_nndescent(_ptr(X), n, d, d, K, S, max_iters, int(stop_updates),
                             ctypes.c_uint64(seed & (2**64 - 1)), _ptr(ids), _ptr(d2),
                             _ptr(flags), _ptr(stats)), "nndescent")
    it = int(stats[0])
    return ids, d2, flags, {"iters": it,
                            "updates": [int(x) for x in stats[1:1 + 2 * it:2]],
                            "pairs": [int(x) for x in stats[2:2 + 2 * it:2]]}


def prune_one(X, u, cand, R, alpha_deg=60.0, strict_ties=False, force_angle=False):
    """Alg. 3 (with the alpha test) for one node; returns kept ids and d2."""
    lib = _load()
    X = _f32(X)
    cand = _i32(cand)
    ids = np.empty(R, np.int32)
    d2 = np.empty(R, np.float64)
    k = lib.orc_prune_one(_ptr(X), X.shape[1], X.shape[1], int(u), _ptr(cand), len(cand), R,
                          float(alpha_deg), int(bool(strict_ties)), int(bool(force_angle)),
                          _ptr(ids), _ptr(d2))
    if k < 0:
        raise RuntimeError(f"oracle prune_one failed with status {k}")
    return ids[:k].copy(), d2[:k].copy()


def prune_table(cand, tab, R, alpha_deg=60.0, strict_ties=False):
    """Prune every node with all distances read from tab (n, C+1, C+1) float32."""
    lib = _load()
    cand = _i32(cand)
    n, C = cand.shape
    tab = _f32(tab)
    assert tab.shape == (n, C + 1, C + 1)
    ids = np.empty((n, R), np.int32)
    d2 = np.empty((n, R), np.float64)
    deg = np.empty(n, np.int32)
    _check(lib.orc_prune_table(n, _ptr(cand), C, _ptr(tab), R, float(alpha_deg),
                               int(bool(strict_ties)), _ptr(ids), _ptr(d2), _ptr(deg)),
           "prune_table")
    return ids, d2, deg


def entry_point(X):
    X = _f32(X)
    r = _load().orc_entry_point(_ptr(X), X.shape[0], X.shape[1], X.shape[1])
    if r < 0:
        raise RuntimeError(f"oracle entry_point failed with status {r}")
    return int(r)


def refine(X, cand, R, alpha_deg=60.0, strict_ties=False, stages=STAGES_ALL):
    """Alg. 2 Phase 3 on candidate lists; returns dict(ids, d2, deg, ep, roots)."""
    lib = _load()
    X = _f32(X)
    cand = _i32(cand)
    n, d = X.shape
    C = cand.shape[1]
    ids = np.empty((n, R), np.int32)
    d2 = np.empty((n, R), np.float64)
    deg = np.empty(n, np.int32)
    ep = np.zeros(1, np.int32)
    roots = np.empty(n, np.int32)
    nroots = np.zeros(1, np.int32)
    _check(lib.orc_refine(_ptr(X), n, d, d, _ptr(cand), C, R, float(alpha_deg),
                          int(bool(strict_ties)), stages, _ptr(ids), _ptr(d2), _ptr(deg),
                          _ptr(ep), _ptr(roots), _ptr(nroots)), "refine")
    return {"ids": ids, "d2": d2, "deg": deg, "ep": int(ep[0]),
            "roots": roots[:int(nroots[0])].copy()}


def search(X, g_ids, g_deg, Q, entries, k, L):
    """Alg. 1 beam search from a set of entering points; returns ids, d2, stats (nq, 2)."""
    lib = _load()
    X, Q = _f32(X), _f32(Q)
    g_ids, g_deg, entries = _i32(g_ids), _i32(g_deg), _i32(np.atleast_1d(entries))
    n, d = X.shape
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.int32)
    d2 = np.empty((nq, k), np.float64)
    stats = np.empty((nq, 2), np.int64)
    _check(lib.orc_search(_ptr(X), n, d, d, _ptr(g_ids), g_ids.shape[1], _ptr(g_deg),
                          _ptr(Q), nq, d, _ptr(entries), len(entries), k, L,
                          _ptr(ids), _ptr(d2), _ptr(stats)), "search")
    return ids, d2, stats


def search_self(X, g_ids, g_deg, k, L):
    """Alg. 5 Phase 3: KANNSearch(G, u, k, L, u) for every u, u itself left out."""
    lib = _load()
    X = _f32(X)
    g_ids, g_deg = _i32(g_ids), _i32(g_deg)
    n, d = X.shape
    ids = np.empty((n, k), np.int32)
    d2 = np.empty((n, k), np.float64)
    stats = np.empty((n, 2), np.int64)
    _check(lib.orc_search_self(_ptr(X), n, d, d, _ptr(g_ids), g_ids.shape[1], _ptr(g_deg), k, L,
                               _ptr(ids), _ptr(d2), _ptr(stats)), "search_self")
    return ids, d2, stats


def opt_kcna(X, cand, k, L, M, alpha_deg):
    """OptKCNA (Alg. 5): the alpha-PG of the candidate lists (prune with M and
    alpha, reverse re-prune, connect), then a search from every point on it.
    Returns the new candidate lists (n x k) and their d2."""
    g = refine(X, cand, M, alpha_deg=alpha_deg)
    ids, d2, _ = search_self(X, g["ids"], g["deg"], k, L)
    return ids, d2


def quality_sample_size(n, eps, l=1):
    """Sample size of the quality examination (Section 5.2, the theorem on
    n_s): n_s >= (8 + 2 eps) l log n / eps^2 (natural log) samples estimate the
    mean k-CNA recall within eps/2 with probability at least 1 - n^-l."""
    return int(math.ceil((8.0 + 2.0 * eps) * l * math.log(n) / (eps * eps)))


def quality_examination(X, cand, k, sample):
    """Estimated k-CNA quality of the candidate lists: the mean over the sampled
    nodes u of |C(u)[:k] & N*_k(u)| / k, with N*_k(u) the exact k nearest other
    points (brute force)."""
    X = _f32(X)
    sample = _i32(sample)
    gt, _ = exact_knn(X, X[sample], k, exclude=sample)
    cand = np.asarray(cand)
    hits = 0
    for u, t in zip(sample.tolist(), gt.tolist()):
        hits += len(set(int(v) for v in cand[u, :k] if v >= 0) & set(t))
    return hits / (k * len(sample))


def iter_nsg(X, K, S, max_iters, seed, stop_updates, k, L, M, alpha_deg, iterations,
             target=None, sample=None):
    """IterNSG (Alg. 6): NN-Descent lists (Phase 1), rounds of OptKCNA, then the
    refinement of Alg. 2 (RNG pruning with M, reverse, entry point, connect).
    Without `target` it runs `iterations` rounds.  With `target`, the quality
    examination (Phase 4) on the sampled nodes runs before each round and the
    rounds stop once the estimate reaches `target` (or after `iterations`).
    Returns the graph dict of refine() plus the final candidate lists ("cand"),
    the rounds run ("rounds") and the estimates ("quality")."""
    cand, _, _, _ = nndescent(X, K, S, max_iters, seed, stop_updates=stop_updates)
    rounds, quality = 0, []
    while rounds < iterations:
        if target is not None:
            quality.append(quality_examination(X, cand, k, sample))
            if quality[-1] >= target:
                break
        cand, _ = opt_kcna(X, cand, k, L, M, alpha_deg)
        rounds += 1
    g = refine(X, cand, M)
    g["cand"], g["rounds"], g["quality"] = cand, rounds, quality
    return g


def recall_at_k(found_ids, true_ids):
    """Recall@k of Section 6: |N*(q) & N(q)| / k averaged over queries."""
    found_ids = np.asarray(found_ids)
    true_ids = np.asarray(true_ids)
    k = true_ids.shape[1]
    hits = 0
    for f, t in zip(found_ids, true_ids):
        hits += len(set(int(x) for x in f[:k] if x >= 0) & set(int(x) for x in t))
    return hits / (k * len(true_ids))


# ------------------------------------------------------------------ OptHNSW (Alg. 7)

def hnsw_levels(U, M):
    """Highest layer of each node, as HNSW draws it (Alg. 7, first loop):
    floor(-ln U / ln M) for U in (0, 1].  Evaluated as the number of i >= 1
    with U * M^i <= 1, M^i being an exact integer in double precision, so no
    logarithm enters.  Levels stop at 31 and at the last i with M^i below
    2^53 (U would have to be below 2^-53 to reach it)."""
    U = np.asarray(U, dtype=np.float64)
    out = np.zeros(len(U), np.int32)
    for j, u in enumerate(U.tolist()):
        lev, p = 0, float(M)
        while lev < 31 and u * p <= 1.0 and p < 2.0 ** 53:
            lev += 1
            p *= M
        out[j] = lev
    return out


def opt_hnsw(X, U, k0, ef, M, alpha_deg, iterations, S, max_iters, seed, delta):
    """OptHNSW (Alg. 7).  D_i = nodes whose highest layer is at least i.  A
    layer with at most M nodes links every node to all the others ((d2, id)
    order); a larger one is IterNSG(D_i, k0, ef, ef, M, alpha) on its rows,
    with NN-Descent K = min(k0, |D_i| - 1), S capped at K, the stop rule
    delta |D_i| K, and C(u) the ef - 1 entries other than u of a pool of
    width ef.  The entry point is the smallest id of the top layer.  Returns
    levels, max_level, ep and per layer: nodes (global ids, ascending), ids
    and deg (local ids)."""
    X = _f32(X)
    levels = hnsw_levels(U, M)
    top = int(levels.max())
    layers = []
    for i in range(top + 1):
        nodes = np.nonzero(levels >= i)[0].astype(np.int32)
        m = len(nodes)
        Xi = X[nodes]
        if m <= M:
            ids = np.full((m, M), -1, np.int32)
            if m >= 2:
                nb, _ = exact_knn(Xi, Xi, m - 1, exclude=np.arange(m, dtype=np.int32))
                ids[:, :m - 1] = nb
            deg = np.full(m, m - 1, np.int32)
        else:
            K = min(k0, m - 1)
            Si = min(S, K)
            g = iter_nsg(Xi, K, Si, max_iters, seed, int(delta * m * K), ef - 1, ef, M, alpha_deg,
                         iterations)
            ids, deg = g["ids"], g["deg"]
        layers.append({"nodes": nodes, "ids": ids, "deg": deg})
    return {"levels": levels, "max_level": top, "ep": int(layers[top]["nodes"][0]), "layers": layers}


def hnsw_search(X, H, Q, k, ef):
    """Greedy routing (KANNSearch with k = L = 1) from the entry point down to
    layer 1, each layer entered at the node found above it, then KANNSearch
    with L = ef on layer 0; one query at a time."""
    X, Q = _f32(X), _f32(Q)
    nq = len(Q)
    ids = np.empty((nq, k), np.int32)
    d2 = np.empty((nq, k), np.float64)
    for q in range(nq):
        w = H["ep"]
        for i in range(H["max_level"], 0, -1):
            lay = H["layers"][i]
            local = int(np.searchsorted(lay["nodes"], w))
            r, _, _ = search(X[lay["nodes"]], lay["ids"], lay["deg"], Q[q:q + 1],
                             np.array([local], np.int32), 1, 1)
            w = int(lay["nodes"][r[0, 0]])
        lay = H["layers"][0]
        r, rd, _ = search(X, lay["ids"], lay["deg"], Q[q:q + 1], np.array([w], np.int32), k, ef)
        ids[q], d2[q] = r[0], rd[0]
    return ids, d2
