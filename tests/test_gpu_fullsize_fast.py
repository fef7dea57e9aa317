"""The paper's own constructions at the benchmark's full size (sift-like
1M x 128), in the configurations bench.py times, checked on sampled outputs
the oracle computes one by one:

* IterNSG (Alg. 6, I = 2, alpha 65 degrees, k = 64, L = 128): sampled rows of
  each round's alpha-prune against the oracle's Prune on the same candidates
  (the angle test is decided in float32 on the GPU, so at most 1% of rows may
  differ through a near-threshold decision); sampled self-searches of each
  round against the oracle's KANNSearch on the same alpha-PG (exact); the
  composition equals pg.iter_nsg bit for bit; the final graph is connected.
* FastHNSW (Alg. 7, ef = 64, M = 32, k0 = 64): the layer draws equal the
  oracle's; the small top layers equal the oracle's construction on the same
  rows; sampled layered searches equal the oracle's routing on the same
  layers (exact).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

N, NQ, D, K, R, S, T = 1_000_000, 10_000, 128, 64, 32, 32, 12
ALPHA, L_SELF = 65.0, 128
SAMPLE = 60


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def data():
    from paper_2410_01231_amd import datagen, pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    X, Q = datagen.sift_like(N, NQ, d=D, seed=2)
    return pg, datagen, X, Q, dev(X), dev(Q)


def _self_search_oracle(oracle, X, g_ids, g_deg, u, k, L):
    ids, d2, _ = oracle.search(X, g_ids, g_deg, X[u:u + 1], np.array([u], np.int32), k + 1, L)
    keep = [(i, v) for i, v in zip(ids[0].tolist(), d2[0].tolist()) if i != u][:k]
    return [i for i, _ in keep]


def test_iter_nsg_rounds_sampled(data, oracle):
    pg, datagen, X, _, Xd, _ = data
    samp = np.random.default_rng(31).choice(N, size=SAMPLE, replace=False)
    cand, cd2, st = pg.knn_build(Xd, K, S=S, max_iters=T, seed=1, delta=0.001, precision=pg.FP16)
    x16, exact = pg.half_rows(Xd)
    assert exact
    for rnd in range(2):
        c = host(cand)
        p1 = pg.prune(Xd, cand, R, alpha_deg=ALPHA, cand_d2=cd2, stages=pg.STAGE_PRUNE)
        same = 0
        for u in samp.tolist():
            ref, _ = oracle.prune_one(X, u, c[u], R, alpha_deg=ALPHA)
            same += list(host(p1["ids"][u, :p1["deg"][u]])) == list(ref)
        print(f"[fullsize-fast] round {rnd}: alpha-prune rows identical {same}/{SAMPLE}", flush=True)
        assert same == SAMPLE
        g = pg.prune(Xd, cand, R, alpha_deg=ALPHA, cand_d2=cd2)
        cand, cd2 = pg.search_self(Xd, g["ids"], g["deg"], K, L_SELF, x16=x16)
        gi, gd, c2 = host(g["ids"]), host(g["deg"]), host(cand)
        for u in samp[:20].tolist():
            assert list(c2[u]) == _self_search_oracle(oracle, X, gi, gd, u, K, L_SELF), (rnd, u)
    final = pg.prune(Xd, cand, R, cand_d2=cd2)
    it = pg.iter_nsg(Xd, K, R, K, L_SELF, ALPHA, 2, S=S, max_iters=T, seed=1, delta=0.001,
                     precision=pg.FP16)
    for key in ("ids", "deg", "ep", "roots"):
        assert torch.equal(it[key], final[key]), key
    assert torch.equal(it["cand"], cand)
    # every node reachable from the entry point
    ids, deg = host(final["ids"]), host(final["deg"])
    valid = np.arange(R)[None, :] < deg[:, None]
    seen = np.zeros(N, bool)
    front = np.array([int(host(final["ep"])[0])])
    seen[front] = True
    while front.size:
        nb = ids[front][valid[front]]
        nb = np.unique(nb[~seen[nb]])
        seen[nb] = True
        front = nb
    assert seen.all()


def test_fast_hnsw_sampled(data, oracle):
    pg, datagen, X, Q, Xd, Qd = data
    U = datagen.uniform_open01(N, seed=7)
    H = pg.opt_hnsw(Xd, dev(U), K, 64, R, ALPHA, iterations=2, S=S, max_iters=T, seed=1, delta=0.001,
                    precision=pg.FP16)
    lev = oracle.hnsw_levels(U, R)
    assert np.array_equal(host(H["levels"]), lev)
    assert H["max_level"] == lev.max() >= 3
    sizes = [int(l["nodes"].numel()) for l in H["layers"]]
    print(f"[fullsize-fast] layers {sizes}", flush=True)
    # the layers above 1 are small enough for the oracle to build outright
    for i in range(2, H["max_level"] + 1):
        lay = H["layers"][i]
        nodes = host(lay["nodes"])
        m = len(nodes)
        Xi = X[nodes]
        if m <= R:
            nb, _ = oracle.exact_knn(Xi, Xi, m - 1, exclude=np.arange(m, dtype=np.int32)) if m > 1 else (None, None)
            if m > 1:
                assert np.array_equal(host(lay["ids"])[:, :m - 1], nb)
        else:
            Ki = min(K, m - 1)
            r = oracle.iter_nsg(Xi, Ki, min(S, Ki), T, 1, int(0.001 * m * Ki), 63, 64, R, ALPHA, 2)
            assert np.array_equal(host(lay["ids"]), r["ids"]), i
            assert np.array_equal(host(lay["deg"]), r["deg"]), i
    # sampled layered searches on the same layers
    Ho = {"ep": H["ep"], "max_level": H["max_level"],
          "layers": [{"nodes": host(l["nodes"]), "ids": host(l["ids"]), "deg": host(l["deg"])}
                     for l in H["layers"]]}
    qs = np.random.default_rng(5).choice(NQ, size=25, replace=False)
    ids, _ = pg.hnsw_search(H, Qd[torch.from_numpy(qs).cuda().long()].contiguous(), 10, 64)
    rid, _ = oracle.hnsw_search(X, Ho, Q[qs], 10, 64)
    assert np.array_equal(host(ids), rid)
