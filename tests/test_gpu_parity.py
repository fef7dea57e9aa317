"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Integer-valued data makes every float32 squared distance exact (all partial
sums are integers below 2^24), so on it the two sides must agree bit for bit:
distances, kNN lists, NN-Descent counters, prune edge sets, entry point,
connect roots and search results.  On float data the distances must agree to
1e-5 relative and whole-graph results statistically.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg():
    from paper_2410_01231_amd import pg as _pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _pg.load_library()
    return _pg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def log(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------- exact kNN
@pytest.mark.parametrize("n,d,k", [(3000, 128, 10), (777, 96, 64), (65, 4, 1)])
def test_exact_knn_bit_exact(pg, oracle, datagen, n, d, k):
    log("exact_knn", n, d, k)
    X = datagen.uniform_int(n, d, seed=n)
    Q = datagen.uniform_int(123, d, seed=n + 1)
    ids, d2 = pg.exact_knn(dev(X), dev(Q), k)
    rid, rd2 = oracle.exact_knn(X, Q, k)
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d2), rd2.astype(np.float32))
    # data as its own queries, each skipping itself
    ex = np.arange(200, dtype=np.int32)
    ids, d2 = pg.exact_knn(dev(X), dev(X[:200]), k, exclude=dev(ex))
    rid, rd2 = oracle.exact_knn(X, X[:200], k, exclude=ex)
    assert np.array_equal(host(ids), rid)


def test_exact_knn_float_tolerance(pg, oracle, datagen):
    X, Q = datagen.gist_like(1500, 40, d=960, seed=3)
    ids, d2 = pg.exact_knn(dev(X), dev(Q), 10)
    rid, rd2 = oracle.exact_knn(X, Q, 10)
    g = host(d2).astype(np.float64)
    assert np.max(np.abs(g - rd2) / rd2) < 1e-5
    # ids may differ only where the two candidates' true distances are within tolerance
    same = host(ids) == rid
    assert same.mean() > 0.99


# ---------------------------------------------------------------- NN-Descent
def _knn_oracle(oracle, X, K, S, T, seed, stop):
    return oracle.nndescent(X, K, S, T, seed, stop_updates=stop)


PATHS = {0: "fp32-mfma", 3: "fp32-valu", 1: "fp16-mfma", 2: "bf16-mfma"}


@pytest.mark.parametrize("prec", [0, 3, 1, 2], ids=lambda p: PATHS[p])
@pytest.mark.parametrize("n,d,K,S,T", [(1500, 32, 16, 8, 5), (700, 12, 8, 4, 6), (90, 8, 64, 32, 3),
                                       (600, 40, 24, 12, 4)])
def test_nndescent_bit_exact(pg, oracle, datagen, n, d, K, S, T, prec):
    # integer data in [0, 255]: FP32, FP16 and BF16 MFMA norm expansions are all exact
    log("nndescent", n, d, K, S, T, PATHS[prec])
    X = datagen.uniform_int(n, d, seed=7)
    ids, d2, st = pg.knn_build(dev(X), K, S=S, max_iters=T, seed=5, stop_updates=-1, precision=prec)
    assert st["join_path"] == PATHS[prec]
    rid, rd2, _, rst = _knn_oracle(oracle, X, K, S, T, 5, -1)
    assert st["updates"] == rst["updates"]
    assert st["pairs"] == rst["pairs"]
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d2), rd2.astype(np.float32))


@pytest.mark.parametrize("prec", [0, 3, 1], ids=lambda p: PATHS[p])
def test_nndescent_tuning_knobs_do_not_change_result(pg, datagen, prec):
    # bucket capacity and pass boundaries change speed only: tiny buckets force
    # the spill list and the repeat passes, many passes split every iteration
    X = datagen.uniform_int(2000, 16, seed=11)
    base = pg.knn_build(dev(X), 16, S=8, max_iters=6, seed=3, stop_updates=-1, precision=prec)
    for cap, ch in [(32, 1), (32, 7), (64, 200), (512, 2), (128, 1)]:
        ids, d2, st = pg.knn_build(dev(X), 16, S=8, max_iters=6, seed=3, stop_updates=-1,
                                   bucket_cap=cap, chunks=ch, precision=prec)
        assert torch.equal(ids, base[0]) and torch.equal(d2, base[1]), (cap, ch)
        assert st["updates"] == base[2]["updates"]
        if cap == 32:
            assert st["spilled"] > 0


def test_nndescent_c1_config(pg, oracle, datagen):
    # tiny config: 10,000 x 128 integers, K = 32, S = 16, delta = 0.001
    X = datagen.uniform_int(10000, 128, seed=0)
    stop = int(0.001 * 10000 * 32)
    ids, d2, st = pg.knn_build(dev(X), 32, S=16, max_iters=12, seed=1, stop_updates=stop)
    rid, rd2, _, rst = _knn_oracle(oracle, X, 32, 16, 12, 1, stop)
    log("c1 iters", st["iters"], st["updates"])
    assert st["updates"] == rst["updates"]
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d2), rd2.astype(np.float32))


@pytest.mark.parametrize("gen,prec", [("gist", 1), ("gist", 2), ("deep", 1), ("deep", 2)])
def test_mixed_precision_lists_equal_fp32(pg, datagen, gen, prec):
    # float data: 16-bit tiles on centred data only prefilter; with the
    # rigorous margin every decision and every stored distance is the FP32
    # direct form, so the lists equal the FP32 build bit for bit
    if gen == "gist":
        X, _ = datagen.gist_like(4000, 0, d=240, n_clusters=12, seed=6)
    else:
        X, _ = datagen.unit_mixture(4000, 0, d=96, n_clusters=40, seed=7)
    Xd = dev(X)
    a_ids, a_d2, a_st = pg.knn_build(Xd, 24, S=12, max_iters=6, seed=5, precision=prec)
    b_ids, b_d2, b_st = pg.knn_build(Xd, 24, S=12, max_iters=6, seed=5, precision=pg.FP32)
    log(gen, a_st["join_path"], "rechecked", a_st["rechecked"], "pairs", a_st["pairs"])
    assert a_st["join_path"] == ("fp16-mixed" if prec == 1 else "bf16-mixed")
    assert b_st["join_path"] == "fp32-valu"
    assert torch.equal(a_ids, b_ids)
    assert torch.equal(a_d2, b_d2)
    assert a_st["updates"] == b_st["updates"]
    assert 0 < sum(a_st["rechecked"]) < sum(a_st["pairs"])


def test_mixed_precision_stated_margin_keeps_direct_distances(pg, datagen):
    # margin_rel < 0: the stated relative margin alone (not rigorous).  Stored
    # distances are still the direct form, so each entry's d2 equals the FP32
    # build's value for the same pair wherever both lists hold it.
    X, _ = datagen.gist_like(3000, 0, d=240, n_clusters=12, seed=8)
    Xd = dev(X)
    a_ids, a_d2, a_st = pg.knn_build(Xd, 16, S=8, max_iters=5, seed=2, precision=pg.FP16,
                                     margin_rel=-1e-3)
    b_ids, b_d2, _ = pg.knn_build(Xd, 16, S=8, max_iters=5, seed=2, precision=pg.FP32)
    ai, ad, bi, bd = host(a_ids), host(a_d2), host(b_ids), host(b_d2)
    assert (np.diff(ad, axis=1) >= 0).all()
    common = 0
    for u in range(len(X)):
        m = dict(zip(bi[u].tolist(), bd[u].tolist()))
        for v, dv in zip(ai[u].tolist(), ad[u].tolist()):
            if v in m:
                assert m[v] == dv
                common += 1
    assert common > 0.9 * ai.size


def test_nndescent_float_statistical(pg, oracle, datagen):
    X, _ = datagen.unit_mixture(4000, 0, d=96, n_clusters=40, seed=4)
    ids, d2, st = pg.knn_build(dev(X), 16, S=8, max_iters=10, seed=2)
    assert st["join_path"] == "fp32-valu"  # norm expansion is not exact on this data
    with pytest.raises(pg.PgError) as e:
        pg.knn_build(dev(X), 16, S=8, max_iters=2, seed=2, precision=pg.FP16, margin_rel=2.0)
    assert e.value.status == -1
    rid, rd2, _, rst = oracle.nndescent(X, 16, 8, 10, 2, stop_updates=int(0.001 * 4000 * 16))
    gt, _ = oracle.exact_knn(X, X, 16, exclude=np.arange(4000))
    g = host(ids)

    def rec(a):
        return np.mean([len(set(x) & set(y)) / 16 for x, y in zip(a, gt)])
    rg, ro = rec(g), rec(rid)
    log("float knn recall gpu", rg, "oracle", ro)
    assert abs(rg - ro) < 0.01 and rg > 0.9
    # stored distances are the float32 distances of the listed pairs
    Xd = X.astype(np.float64)
    for u in range(0, 4000, 97):
        true = ((Xd[g[u]] - Xd[u]) ** 2).sum(1)
        assert np.max(np.abs(host(d2)[u] - true) / np.maximum(true, 1e-30)) < 1e-5


# ---------------------------------------------------------------- prune
def _exact_lists(oracle, X, K):
    ids, _ = oracle.exact_knn(X, X, K, exclude=np.arange(len(X)))
    return ids


@pytest.mark.parametrize("alpha,strict", [(60.0, False), (60.0, True)])
def test_prune_stage_bit_exact(pg, oracle, datagen, alpha, strict):
    X = datagen.uniform_int(1200, 32, seed=2)
    cand = _exact_lists(oracle, X, 24)
    g = pg.prune(dev(X), dev(cand), 12, alpha_deg=alpha, strict_ties=strict, stages=pg.STAGE_PRUNE)
    r = oracle.refine(X, cand, 12, alpha_deg=alpha, strict_ties=strict, stages=oracle.STAGE_PRUNE)
    assert np.array_equal(host(g["deg"]), r["deg"])
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert np.array_equal(host(g["d2"]), r["d2"].astype(np.float32))


def test_prune_candidates_with_repeats_self_and_padding(pg, oracle, datagen):
    X = datagen.uniform_int(500, 8, seed=4)
    cand = datagen.random_candidates(500, 40, seed=4)
    cand[:, 5] = np.arange(500)          # self
    cand[:, 7] = cand[:, 6]              # repeat
    cand[::3, 9] = -1                    # padding
    g = pg.prune(dev(X), dev(cand), 10, stages=pg.STAGE_PRUNE)
    r = oracle.refine(X, cand, 10, stages=oracle.STAGE_PRUNE)
    assert np.array_equal(host(g["ids"]), r["ids"])


def test_full_refine_bit_exact(pg, oracle, datagen):
    # clustered integer data: the pruned graph is disconnected, connect must add edges
    X, _ = datagen.sift_like(3000, 0, d=32, n_clusters=20, sigma=6.0, seed=8)
    cand = _exact_lists(oracle, X, 32)
    g = pg.prune(dev(X), dev(cand), 16)
    r = oracle.refine(X, cand, 16)
    log("roots gpu", len(g["roots"]), "oracle", len(r["roots"]))
    assert int(host(g["ep"])[0]) == r["ep"]
    assert np.array_equal(host(g["roots"]), r["roots"])
    assert np.array_equal(host(g["deg"]), r["deg"])
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert len(r["roots"]) > 0


@pytest.mark.parametrize("nn,d,nc,sigma,C,R,seed", [
    (1200, 16, 12, 4.0, 10, 3, 14),   # small R: many candidates saturate, exact scans
    (2500, 8, 40, 1.5, 6, 4, 21),     # many tight clusters: roots with no reached candidate
])
def test_connect_saturation_bit_exact(pg, oracle, datagen, nn, d, nc, sigma, C, R, seed):
    X, _ = datagen.sift_like(nn, 0, d=d, n_clusters=nc, sigma=sigma, seed=seed)
    cand = _exact_lists(oracle, X, C)
    g = pg.prune(dev(X), dev(cand), R)
    r = oracle.refine(X, cand, R)
    log("roots gpu", len(g["roots"]), "oracle", len(r["roots"]))
    assert len(r["roots"]) > 20
    assert np.array_equal(host(g["roots"]), r["roots"])
    assert np.array_equal(host(g["deg"]), r["deg"])
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert np.array_equal(host(g["d2"]), r["d2"].astype(np.float32))


@pytest.mark.parametrize("R", [8, 12])
def test_connect_alpha_graph_bit_exact(pg, oracle, datagen, R):
    # alpha = 65 on exact lists in 128 dimensions: after the reverse re-prune
    # almost every node sits at degree R, so most roots have no usable
    # candidate and take the nearest free node of the whole graph (at R = 8
    # there are more roots than free nodes)
    X, _ = datagen.sift_like(8000, 0, d=128, n_clusters=80, sigma=20.0, seed=31)
    cand = _exact_lists(oracle, X, 32)
    g = pg.prune(dev(X), dev(cand), R, alpha_deg=65.0)
    r = oracle.refine(X, cand, R, alpha_deg=65.0)
    log("roots gpu", len(g["roots"]), "oracle", len(r["roots"]))
    assert len(r["roots"]) > 200
    assert np.array_equal(host(g["roots"]), r["roots"])
    assert np.array_equal(host(g["deg"]), r["deg"])
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert np.array_equal(host(g["d2"]), r["d2"].astype(np.float32))


def test_connect_alpha_graph_wide_exact_rows_bit_exact(pg, oracle, datagen):
    # exact integer rows of 200 dimensions: the scan over F takes its
    # distances from MFMA tiles with 13 16-dimension steps held in registers
    X, _ = datagen.sift_like(4000, 0, d=200, n_clusters=40, sigma=20.0, seed=37)
    cand = _exact_lists(oracle, X, 24)
    g = pg.prune(dev(X), dev(cand), 12, alpha_deg=65.0)
    r = oracle.refine(X, cand, 12, alpha_deg=65.0)
    log("roots gpu", len(g["roots"]), "oracle", len(r["roots"]))
    assert len(r["roots"]) > 100  # 265 (at R = 8 and 10 both sides report the overflow)
    assert np.array_equal(host(g["roots"]), r["roots"])
    assert np.array_equal(host(g["deg"]), r["deg"])
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert np.array_equal(host(g["d2"]), r["d2"].astype(np.float32))


def test_connect_overflow_is_reported(pg, oracle, datagen):
    # R = 2 on tight clusters: at some turn every reached node has degree R
    X, _ = datagen.sift_like(1500, 0, d=8, n_clusters=30, sigma=2.0, seed=15)
    cand = _exact_lists(oracle, X, 6)
    with pytest.raises(RuntimeError):
        oracle.refine(X, cand, 2)
    with pytest.raises(pg.PgError, match="degree"):
        pg.prune(dev(X), dev(cand), 2)


@pytest.mark.parametrize("nn,d,C,R,alpha,strict,connect", [
    (3000, 48, 40, 12, 60.0, False, True),    # one partial dimension chunk
    (3000, 132, 40, 12, 67.0, False, False),  # chunks of 64, 64, 16; alpha test (connect
                                              # would overflow here, on both sides)
    (2500, 64, 32, 10, 60.0, True, True),     # strict ties
    (2000, 32, 64, 40, 60.0, False, True),    # reverse unions above 64: several rounds
])
def test_prune_mfma_exact_path_bit_exact(pg, oracle, datagen, nn, d, C, R, alpha, strict, connect):
    # integer data and given candidate distances: pairwise distances come from
    # FP16 MFMA Gram tiles, which are exact here
    X, _ = datagen.sift_like(nn, 0, d=d, n_clusters=20, sigma=6.0, seed=31)
    cand, cd2 = oracle.exact_knn(X, X, C, exclude=np.arange(nn))
    st_g = pg.STAGES_ALL if connect else pg.STAGE_PRUNE | pg.STAGE_REVERSE
    st_o = oracle.STAGE_PRUNE | oracle.STAGE_REVERSE | (oracle.STAGE_CONNECT if connect else 0)
    g = pg.prune(dev(X), dev(cand), R, alpha_deg=alpha, strict_ties=strict, stages=st_g,
                 cand_d2=dev(cd2.astype(np.float32)))
    r = oracle.refine(X, cand, R, alpha_deg=alpha, strict_ties=strict, stages=st_o)
    log("roots gpu", len(g["roots"]), "oracle", len(r["roots"]))
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert np.array_equal(host(g["deg"]), r["deg"])
    assert np.array_equal(host(g["d2"]), r["d2"].astype(np.float32))
    assert np.array_equal(host(g["roots"]), r["roots"])
    assert int(host(g["ep"])[0]) == r["ep"]


def test_prune_mfma_unsorted_candidates_with_repeats(pg, oracle, datagen):
    # the exact MFMA path on candidate lists that are not kNN lists: random
    # order, repeats, u itself and -1 padding, with their exact distances given
    X, _ = datagen.sift_like(1500, 0, d=40, n_clusters=10, sigma=8.0, seed=33)
    n = len(X)
    cand = datagen.random_candidates(n, 48, seed=34)
    cand[:, 5] = cand[:, 2]              # repeats
    cand[::7, 9] = np.arange(n)[::7]     # self
    cand[::3, 47] = -1                   # padding
    Xd64 = X.astype(np.float64)
    safe = np.where(cand >= 0, cand, 0)
    cd2 = ((Xd64[:, None, :] - Xd64[safe]) ** 2).sum(-1).astype(np.float32)
    g = pg.prune(dev(X), dev(cand), 16, cand_d2=dev(cd2), stages=pg.STAGE_PRUNE | pg.STAGE_REVERSE)
    r = oracle.refine(X, cand, 16, stages=oracle.STAGE_PRUNE | oracle.STAGE_REVERSE)
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert np.array_equal(host(g["deg"]), r["deg"])


def test_prune_given_distances_match_computed_on_float_data(pg, datagen):
    # non-integer data keep the canonical FP32 path; given distances from the
    # kNN build are the same chain values, so the graphs are identical
    X, _ = datagen.gist_like(1500, 0, d=64, n_clusters=10, seed=5)
    Xd = dev(X)
    ids, d2, _ = pg.knn_build(Xd, 24, S=12, max_iters=1, seed=3, exact=True)
    a = pg.prune(Xd, ids, 12, cand_d2=d2)
    b = pg.prune(Xd, ids, 12)
    for k in ("ids", "d2", "deg", "roots", "ep"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("law,alpha,strict", [("gist", 60.0, False), ("gist", 65.0, False),
                                               ("deep", 60.0, True), ("deep", 89.0, False),
                                               ("sift", 60.0, False), ("sift", 120.0, False),
                                               ("gist512", 60.0, False), ("gist512", 89.0, True)])
def test_prune_mixed_tiles_equal_chains_on_float_data(pg, datagen, law, alpha, strict):
    # float data: the MFMA prune on the centred FP16 copy decides only what
    # its error bound allows and takes the FP32 chain for the rest, so its
    # graph equals the all-chain prune, for every stage (the reverse unions
    # run on both kernels too); duplicated rows give zero distances and ties.
    # Rows of 256 dimensions or more take their chains from rows staged
    # through LDS (gist512), shorter ones stream them per lane.
    log("mixed prune", law, alpha, strict)
    if law == "gist512":
        X, _ = datagen.gist_like(2500, 0, d=512, n_clusters=10, seed=8)
    elif law == "gist":
        X, _ = datagen.gist_like(3000, 0, d=240, n_clusters=10, seed=5)
    elif law == "deep":
        X, _ = datagen.unit_mixture(4000, 0, d=96, n_clusters=20, seed=6)
    else:
        X, _ = datagen.sift_like(3000, 0, d=128, n_clusters=20, seed=7)
        X = X * np.float32(0.37) + np.float32(0.011)
    X = np.ascontiguousarray(X)
    X[200:260] = X[0:60]
    Xd = dev(X)
    ids, d2, _ = pg.knn_build(Xd, 48, S=24, max_iters=6, seed=2)
    # the prune stages (connect may overflow at wide angles on clustered data)
    st = pg.STAGE_PRUNE | pg.STAGE_REVERSE
    a = pg.prune(Xd, ids, 24, alpha_deg=alpha, strict_ties=strict, cand_d2=d2, stages=st)
    b = pg.prune(Xd, ids, 24, alpha_deg=alpha, strict_ties=strict, cand_d2=d2, precision=pg.FP32_VALU,
                 stages=st)
    for k in ("ids", "d2", "deg", "ep"):
        assert torch.equal(a[k], b[k]), k


def test_prune_table_hook_float_bit_exact(pg, oracle, datagen):
    # identical candidate lists and identical float32 distances -> identical edges
    X, _ = datagen.unit_mixture(400, 0, d=16, n_clusters=5, seed=6)
    C = 20
    cand = datagen.random_candidates(400, C, seed=6)
    for u in range(400):  # distinct ids, not u
        row = np.unique(cand[u][cand[u] != u])
        extra = np.setdiff1d(np.arange(400), np.append(row, u))[: C - len(row)]
        cand[u] = np.concatenate([row, extra])[:C]
    pos = np.concatenate([np.arange(400)[:, None], cand], 1)
    P = X.astype(np.float64)[pos]
    tab = ((P[:, :, None, :] - P[:, None, :, :]) ** 2).sum(-1).astype(np.float32)
    g = pg.prune(dev(X), dev(cand), 8, stages=pg.STAGE_PRUNE, pair_d2=dev(tab))
    r_ids, r_d2, r_deg = oracle.prune_table(cand, tab, 8)
    assert np.array_equal(host(g["deg"]), r_deg)
    assert np.array_equal(host(g["ids"]), r_ids)


ALPHAS = [62.0, 65.0, 67.0, 89.0, 90.0, 120.0]


@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("data", ["uniform", "grid"])
def test_prune_alpha_bit_exact(pg, oracle, datagen, alpha, data):
    # alpha > 60 on integer data: the distances are exact on both sides and
    # the GPU decides the angle test as the double-precision expression the
    # oracle evaluates (FP32 only outside a proven band), so every row is
    # identical.  The grid data (values 0..3) are full of equal distances and
    # exact right and 120-degree angles, where decisions sit on the threshold.
    # Both prune kernels: canonical chains (no candidate distances given) and
    # the exact FP16 Gram path (given), PRUNE then REVERSE.
    if data == "uniform":
        X = datagen.uniform_int(800, 16, seed=12)
    else:
        X = datagen.int_grid(900, 8, 0, 3, seed=13)
    n = len(X)
    cand, cd2 = oracle.exact_knn(X, X, 24, exclude=np.arange(n, dtype=np.int32))
    st_g = pg.STAGE_PRUNE | pg.STAGE_REVERSE
    r1 = oracle.refine(X, cand, 12, alpha_deg=alpha, stages=oracle.STAGE_PRUNE)
    r2 = oracle.refine(X, cand, 12, alpha_deg=alpha, stages=oracle.STAGE_PRUNE | oracle.STAGE_REVERSE)
    for given in (None, cd2.astype(np.float32)):
        kw = {} if given is None else {"cand_d2": dev(given)}
        g1 = pg.prune(dev(X), dev(cand), 12, alpha_deg=alpha, stages=pg.STAGE_PRUNE, **kw)
        g2 = pg.prune(dev(X), dev(cand), 12, alpha_deg=alpha, stages=st_g, **kw)
        log("alpha", alpha, data, "given" if given is not None else "computed",
            "rows identical", (host(g1["ids"]) == r1["ids"]).all(1).mean(),
            (host(g2["ids"]) == r2["ids"]).all(1).mean())
        assert np.array_equal(host(g1["ids"]), r1["ids"])
        assert np.array_equal(host(g1["deg"]), r1["deg"])
        assert np.array_equal(host(g2["ids"]), r2["ids"])
        assert np.array_equal(host(g2["deg"]), r2["deg"])
        assert np.array_equal(host(g2["d2"]), r2["d2"].astype(np.float32))


def test_prune_alpha_table_hook_bit_exact(pg, oracle, datagen):
    # identical candidate lists and identical float32 distances (the table
    # hook) on float data: the alpha decisions are the same double-precision
    # evaluation on both sides, so the edge sets are identical
    X, _ = datagen.unit_mixture(400, 0, d=16, n_clusters=5, seed=16)
    C = 20
    cand = datagen.random_candidates(400, C, seed=16)
    for u in range(400):
        row = np.unique(cand[u][cand[u] != u])
        extra = np.setdiff1d(np.arange(400), np.append(row, u))[: C - len(row)]
        cand[u] = np.concatenate([row, extra])[:C]
    pos = np.concatenate([np.arange(400)[:, None], cand], 1)
    P = X.astype(np.float64)[pos]
    tab = ((P[:, :, None, :] - P[:, None, :, :]) ** 2).sum(-1).astype(np.float32)
    for alpha in ALPHAS:
        g = pg.prune(dev(X), dev(cand), 8, alpha_deg=alpha, stages=pg.STAGE_PRUNE, pair_d2=dev(tab))
        r_ids, r_d2, r_deg = oracle.prune_table(cand, tab, 8, alpha_deg=alpha)
        assert np.array_equal(host(g["deg"]), r_deg), alpha
        assert np.array_equal(host(g["ids"]), r_ids), alpha


@pytest.mark.parametrize("lo,hi,d", [(-512, 511, 16), (-2048, 2047, 4), (-3, 3, 8)])
def test_signed_integer_paths_identical(pg, oracle, datagen, lo, hi, d):
    # signed integer data: the MFMA norm expansion is exact only while every
    # squared distance stays at or below 2^24.  (-512, 511) in 16 dims passes
    # the test (norms <= 2^22) and takes the MFMA paths; (-2048, 2047) in
    # 4 dims reaches distances near 2^26, where FP32 sums round, and must
    # keep the direct form (the FP16 request then runs the mixed path).
    # Every precision gives the same lists and graph; where every distance is
    # exact they are also the oracle's.
    X = datagen.int_grid(1200, d, lo, hi, seed=lo & 0xFFFF)
    K, S, T, R = 16, 8, 5, 10
    exact = hi < 2047
    if exact:
        ro, rd2, _, _ = oracle.nndescent(X, K, S, T, 5, stop_updates=-1)
        rg = oracle.refine(X, ro, R)
    res = {}
    for prec in (pg.FP32_VALU, pg.FP32, pg.FP16):
        ids, d2, st = pg.knn_build(dev(X), K, S=S, max_iters=T, seed=5, stop_updates=-1, precision=prec)
        g = pg.prune(dev(X), ids, R, cand_d2=d2)
        log("signed", lo, hi, d, "precision", prec, "path", st["join_path"])
        res[prec] = (host(ids), host(d2), host(g["ids"]), host(g["roots"]), st["join_path"])
        if exact:
            assert np.array_equal(res[prec][0], ro), prec
            assert np.array_equal(res[prec][1], rd2.astype(np.float32)), prec
            assert np.array_equal(res[prec][2], rg["ids"]), prec
            assert np.array_equal(res[prec][3], rg["roots"]), prec
    for prec in (pg.FP32, pg.FP16):
        for a, b in zip(res[prec][:4], res[pg.FP32_VALU][:4]):
            assert np.array_equal(a, b), prec
    if exact:
        assert res[pg.FP32][4] == "fp32-mfma" and res[pg.FP16][4] == "fp16-mfma"
    else:
        assert res[pg.FP32][4] == "fp32-valu" and res[pg.FP16][4] == "fp16-mixed"


# ---------------------------------------------------------------- search
def test_search_bit_exact(pg, oracle, datagen):
    X, Q = datagen.sift_like(4000, 299, d=32, n_clusters=10, sigma=10.0, seed=9)
    cand = _exact_lists(oracle, X, 24)
    r = oracle.refine(X, cand, 12)
    entries = np.concatenate([[r["ep"]], r["roots"]]).astype(np.int32)
    for L in (10, 37, 128):
        ids, d2 = pg.search(dev(X), dev(r["ids"]), dev(r["deg"]), dev(Q), dev(entries), 10, L)
        rid, rd2, _ = oracle.search(X, r["ids"], r["deg"], Q, entries, 10, L)
        assert np.array_equal(host(ids), rid), L
        assert np.array_equal(host(d2), rd2.astype(np.float32)), L


def test_search_pools_above_1024_bit_exact(pg, oracle, datagen):
    # pools of 1536 and 2048 on a 2500-node graph: the search takes in most of
    # the graph; FP32 and FP16 rows, both query-per-wave layouts
    X, Q = datagen.sift_like(2500, 37, d=64, n_clusters=6, sigma=14.0, seed=23)
    cand = _exact_lists(oracle, X, 24)
    r = oracle.refine(X, cand, 12)
    entries = np.concatenate([[r["ep"]], r["roots"]]).astype(np.int32)
    x16, exact = pg.half_rows(dev(X))
    assert exact
    for L in (1536, 2048):
        rid, rd2, _ = oracle.search(X, r["ids"], r["deg"], Q, entries, 10, L)
        for rows in (None, x16):
            ids, d2 = pg.search(dev(X), dev(r["ids"]), dev(r["deg"]), dev(Q), dev(entries), 10, L, x16=rows)
            assert np.array_equal(host(ids), rid), L
            assert np.array_equal(host(d2), rd2.astype(np.float32)), L


def test_search_rejects_queries_beyond_lds(pg, datagen):
    # 8192-dimensional rows, a pool of 2048 and a record of 1024 need more
    # than 64 KB of LDS per query: an error, before any launch
    X, Q = datagen.sift_like(300, 3, d=8192, n_clusters=2, sigma=4.0, seed=5)
    g = np.zeros((300, 4), np.int32)
    deg = np.full(300, 4, np.int32)
    rec = (dev(np.full((3, 1024), -1, np.int32)), dev(np.zeros((3, 1024), np.float32)))
    with pytest.raises(pg.PgError, match="LDS"):
        pg.search(dev(X), dev(g), dev(deg), dev(Q), dev(np.array([0], np.int32)), 10, 2048, record=rec)


@pytest.mark.parametrize("R,nq", [(48, 301), (80, 129), (1, 7)])
def test_search_wide_rows_bit_exact(pg, oracle, datagen, R, nq):
    # rows wider than 32 (one query per wave) and wider than 64 (neighbours in
    # chunks); odd query counts leave half a wave without a query
    X, Q = datagen.sift_like(3000, nq, d=32, n_clusters=8, sigma=12.0, seed=17)
    rng = np.random.default_rng(R)
    g = rng.integers(0, 3000, size=(3000, R), dtype=np.int64).astype(np.int32)
    deg = rng.integers(0, R + 1, size=3000).astype(np.int32)
    g[np.arange(R)[None, :] >= deg[:, None]] = -1
    entries = rng.choice(3000, size=70, replace=False).astype(np.int32)
    for L in (16, 100):
        ids, d2 = pg.search(dev(X), dev(g), dev(deg), dev(Q), dev(entries), 10, L)
        rid, rd2, _ = oracle.search(X, g, deg, Q, entries, 10, L)
        assert np.array_equal(host(ids), rid), L
        assert np.array_equal(host(d2), rd2.astype(np.float32)), L


def test_search_fp16_rows_in_large_batches_equal_fp32_rows(pg, oracle, datagen):
    # batches of about 10k queries: the FP16 rows may be staged in 16-
    # dimension slices (when that tile lets the whole launch be resident and
    # the 32-dimension one does not); d = 36 leaves a ragged last slice
    X, Q = datagen.sift_like(4000, 11000, d=36, n_clusters=10, sigma=10.0, seed=19)
    cand = _exact_lists(oracle, X, 24)
    r = oracle.refine(X, cand, 12)
    entries = np.concatenate([[r["ep"]], r["roots"]]).astype(np.int32)
    x16, exact = pg.half_rows(dev(X))
    assert exact
    for nq in (9000, 10000, 11000):
        for L in (64, 192):
            a = pg.search(dev(X), dev(r["ids"]), dev(r["deg"]), dev(Q[:nq]), dev(entries), 10, L, pool_out=True)
            b = pg.search(dev(X), dev(r["ids"]), dev(r["deg"]), dev(Q[:nq]), dev(entries), 10, L, pool_out=True,
                          x16=x16)
            for x, y in zip(a, b):
                assert torch.equal(x, y), (nq, L)
    rid, rd2, _ = oracle.search(X, r["ids"], r["deg"], Q[:300], entries, 10, 192)
    assert np.array_equal(host(b[0][:300]), rid)
    assert np.array_equal(host(b[1][:300]), rd2.astype(np.float32))


def test_search_fp16_rows_equal_fp32_rows(pg, oracle, datagen):
    # an exact FP16 copy of integer data: identical results, pools and
    # counts; float data is reported inexact
    X, Q = datagen.sift_like(4000, 301, d=36, n_clusters=10, sigma=10.0, seed=9)
    cand = _exact_lists(oracle, X, 24)
    r = oracle.refine(X, cand, 12)
    entries = np.concatenate([[r["ep"]], r["roots"]]).astype(np.int32)
    x16, exact = pg.half_rows(dev(X))
    assert exact and tuple(x16.shape) == (4000, 40)
    assert torch.equal(x16[:, :36].float(), dev(X)) and not x16[:, 36:].any()
    for L in (10, 64):
        a = pg.search(dev(X), dev(r["ids"]), dev(r["deg"]), dev(Q), dev(entries), 10, L, pool_out=True)
        b = pg.search(dev(X), dev(r["ids"]), dev(r["deg"]), dev(Q), dev(entries), 10, L, pool_out=True, x16=x16)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        rid, _, _ = oracle.search(X, r["ids"], r["deg"], Q, entries, 10, L)
        assert np.array_equal(host(b[0]), rid)
    # self-search on a wide graph (one query per wave) with FP16 rows
    wide = _exact_lists(oracle, X, 48)
    a = pg.search_self(dev(X), dev(wide), dev(np.full(4000, 48, np.int32)), 8, 20)
    b = pg.search_self(dev(X), dev(wide), dev(np.full(4000, 48, np.int32)), 8, 20, x16=x16)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    Xf, _ = datagen.gist_like(500, 0, d=40, seed=3)
    _, exact = pg.half_rows(dev(Xf))
    assert not exact
    Xb = X.copy()
    Xb[5, 3] = 2049.0  # an integer FP16 cannot hold
    _, exact = pg.half_rows(dev(Xb))
    assert not exact


def test_search_edge_cases(pg, oracle):
    X = np.arange(12, dtype=np.float32).repeat(4).reshape(12, 4)
    g = np.full((12, 2), -1, np.int32)
    deg = np.zeros(12, np.int32)
    for i in range(11):
        g[i, 0] = i + 1
        deg[i] = 1
    Q = np.array([[7.2] * 4, [0.0] * 4], np.float32)
    ent = np.array([0, 0, -1, 3], np.int32)  # repeats and padding
    ids, d2 = pg.search(dev(X), dev(g), dev(deg), dev(Q), dev(ent), 3, 3)
    rid, _, _ = oracle.search(X, g, deg, Q, ent, 3, 3)
    assert np.array_equal(host(ids), rid)
    # L larger than the reachable set: padded output
    ids, d2 = pg.search(dev(X), dev(g), dev(deg), dev(Q), dev(np.array([10], np.int32)), 5, 8)
    assert list(host(ids)[0]) == [10, 11, -1, -1, -1]
    assert np.isinf(host(d2)[0, 2:]).all()


def test_errors_are_reported(pg, datagen):
    X = dev(datagen.uniform_int(50, 8, seed=1))
    with pytest.raises(pg.PgError) as e:
        pg.knn_build(X, 50)  # K >= n
    assert e.value.status == -1
    with pytest.raises(pg.PgError):
        pg.knn_build(X, 8, S=40)
    Xodd = dev(np.zeros((50, 6), np.float32))
    with pytest.raises(pg.PgError) as e:
        pg.knn_build(Xodd, 4)
    assert e.value.status == -4


# ---------------------------------------------------------------- end to end
def test_end_to_end_recall_matches_oracle(pg, oracle, datagen):
    X, Q = datagen.sift_like(6000, 200, d=64, n_clusters=12, seed=21)
    g = pg.build_graph(dev(X), 32, 16, S=16, max_iters=12, seed=4)
    ids_o, _, _, _ = oracle.nndescent(X, 32, 16, 12, 4, stop_updates=int(0.001 * 6000 * 32))
    assert np.array_equal(host(g["knn_ids"]), ids_o)
    r = oracle.refine(X, ids_o, 16)
    assert np.array_equal(host(g["ids"]), r["ids"])
    entries = np.concatenate([[r["ep"]], r["roots"]]).astype(np.int32)
    gt, _ = oracle.exact_knn(X, Q, 10)
    ids, _ = pg.search(dev(X), g["ids"], g["deg"], dev(Q), dev(entries), 10, 64)
    rid, _, _ = oracle.search(X, r["ids"], r["deg"], Q, entries, 10, 64)
    rg, ro = oracle.recall_at_k(host(ids), gt), oracle.recall_at_k(rid, gt)
    log("search recall gpu", rg, "oracle", ro)
    assert abs(rg - ro) <= 0.005


# ------------------------------------------------- OptKCNA / IterNSG (Alg. 5, 6)

def test_search_self_bit_exact(pg, oracle, datagen):
    # the search phase of OptKCNA: every point searched for, entering at itself,
    # itself left out of its own results
    X, _ = datagen.sift_like(2500, 0, d=32, n_clusters=15, sigma=10.0, seed=42)
    cand, _ = oracle.exact_knn(X, X, 20, exclude=np.arange(2500))
    g = oracle.refine(X, cand, 12, alpha_deg=65.0)
    ids, d2 = pg.search_self(dev(X), dev(g["ids"]), dev(g["deg"]), 16, 40)
    rid, rd2, _ = oracle.search_self(X, g["ids"], g["deg"], 16, 40)
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d2), rd2.astype(np.float32))


def test_search_record_reuses_distances_without_changing_results(pg, oracle, datagen):
    # P2K: pools of a search on one graph serve as the record of a search on
    # another graph; the results equal the search without a record (and the
    # oracle's), and part of the distances come from the record
    X, _ = datagen.sift_like(2500, 0, d=32, n_clusters=15, sigma=10.0, seed=42)
    cand, _ = oracle.exact_knn(X, X, 20, exclude=np.arange(2500))
    g1 = oracle.refine(X, cand, 12, alpha_deg=65.0)
    ids1, _ = oracle.search_self(X, g1["ids"], g1["deg"], 16, 40)[:2]
    g2 = oracle.refine(X, ids1, 12, alpha_deg=65.0)
    Xd = dev(X)
    _, _, pi, pd = pg.search_self(Xd, dev(g1["ids"]), dev(g1["deg"]), 16, 40, pool_out=True)
    # a record with padding, a repeat and an out-of-range id must not matter
    pi[:, -1] = -1
    pi[:, -2] = pi[:, 0]
    pd[:, -2] = pd[:, 0]
    pi[::7, -3] = 2500
    c0 = torch.zeros(2, dtype=torch.int64, device="cuda")
    c1 = torch.zeros(2, dtype=torch.int64, device="cuda")
    a = pg.search_self(Xd, dev(g2["ids"]), dev(g2["deg"]), 16, 40, pool_out=True, counts=c0)
    b = pg.search_self(Xd, dev(g2["ids"]), dev(g2["deg"]), 16, 40, record=(pi, pd), pool_out=True,
                       counts=c1)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    rid, rd2, _ = oracle.search_self(X, g2["ids"], g2["deg"], 16, 40)
    assert np.array_equal(host(b[0]), rid)
    assert np.array_equal(host(b[1]), rd2.astype(np.float32))
    c0, c1 = host(c0), host(c1)
    log("computed without record", c0, "with record", c1)
    assert c0[1] == 0 and c1[1] > 0
    assert c1[0] + c1[1] == c0[0]
    assert c1[0] < c0[0]


@pytest.mark.parametrize("nn,d,nc,sig,K,S,k,L,R,alpha", [
    (3000, 32, 20, 12.0, 16, 8, 16, 32, 16, 65.0),
    (2000, 64, 10, 20.0, 24, 12, 24, 40, 20, 62.0),
])
def test_iter_nsg_bit_exact(pg, oracle, datagen, nn, d, nc, sig, K, S, k, L, R, alpha):
    # IterNSG with two OptKCNA rounds, the whole pipeline on integer data
    X, _ = datagen.sift_like(nn, 0, d=d, n_clusters=nc, sigma=sig, seed=41)
    stop = int(0.001 * nn * K)
    g = pg.iter_nsg(dev(X), K, R, k, L, alpha, 2, S=S, max_iters=8, seed=3, stop_updates=stop)
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    gp = pg.iter_nsg(dev(X), K, R, k, L, alpha, 2, S=S, max_iters=8, seed=3, stop_updates=stop, p2k=True,
                     counts=cnt)
    for key in ("ids", "d2", "deg", "ep", "roots", "cand", "cand_d2"):
        assert torch.equal(g[key], gp[key]), key  # P2K leaves the graph unchanged
    log("P2K computed / reused", host(cnt))
    assert host(cnt)[1] > 0
    kc = torch.zeros(2, dtype=torch.int64, device="cuda")
    gk = pg.iter_nsg(dev(X), K, R, k, L, alpha, 2, S=S, max_iters=8, seed=3, stop_updates=stop, k2p=True,
                     k2p_counts=kc)
    for key in ("ids", "d2", "deg", "ep", "roots", "cand", "cand_d2"):
        assert torch.equal(g[key], gk[key]), key  # K2P leaves the graph unchanged
    log("K2P pairs skipped / tested", host(kc))
    assert host(kc)[0] > 0
    r = oracle.iter_nsg(X, K, S, 8, 3, stop, k, L, R, alpha, 2)
    assert np.array_equal(host(g["cand"]), r["cand"])
    assert np.array_equal(host(g["ids"]), r["ids"])
    assert np.array_equal(host(g["deg"]), r["deg"])
    assert np.array_equal(host(g["roots"]), r["roots"])
    assert int(host(g["ep"])[0]) == r["ep"]


@pytest.mark.parametrize("law", ["gist", "deep"])
def test_k2p_on_float_data_leaves_the_graph_unchanged(pg, datagen, law):
    # K2P in the mixed-precision prune (Section 5.4, Exp. 6): skipping the
    # pairs of candidates that both stayed in the previous round's list gives
    # the same graph, three OptKCNA rounds on float data
    if law == "gist":
        X, _ = datagen.gist_like(3000, 0, d=240, n_clusters=10, seed=12)
    else:
        X, _ = datagen.unit_mixture(4000, 0, d=96, n_clusters=20, seed=13)
    Xd = dev(X)
    stop = int(0.001 * len(X) * 24)
    g = pg.iter_nsg(Xd, 24, 32, 24, 48, 65.0, 3, S=12, max_iters=6, seed=2, stop_updates=stop)
    kc = torch.zeros(2, dtype=torch.int64, device="cuda")
    gk = pg.iter_nsg(Xd, 24, 32, 24, 48, 65.0, 3, S=12, max_iters=6, seed=2, stop_updates=stop, k2p=True,
                     k2p_counts=kc)
    for key in ("ids", "d2", "deg", "ep", "roots", "cand", "cand_d2"):
        assert torch.equal(g[key], gk[key]), key
    log(law, "K2P pairs skipped / tested", host(kc))
    assert host(kc)[0] > 0


def test_quality_examination_and_stopping_rule(pg, oracle, datagen):
    # Section 5.2: the sampled k-CNA quality estimate, and IterNSG stopping
    # once it reaches the target, both as in the oracle
    X, _ = datagen.sift_like(3000, 0, d=32, n_clusters=20, sigma=12.0, seed=41)
    n, K, S, k, L, R = len(X), 16, 8, 16, 32, 16
    sample = datagen.sample_ids(n, 300, seed=6)
    cand, _, _, _ = oracle.nndescent(X, K, S, 2, 3)
    assert pg.quality_examination(dev(X), dev(cand), k, sample) == \
        oracle.quality_examination(X, cand, k, sample)
    # per-node counts through the C call, against the oracle's brute force
    est, hits = pg.quality_examination_async(dev(X), dev(cand), 10, sample)
    gt, _ = oracle.exact_knn(X, X[sample], 10, exclude=sample)
    want = [len(set(cand[u, :10].tolist()) & set(t)) for u, t in zip(sample.tolist(), gt.tolist())]
    assert host(hits).tolist() == want
    assert float(est.item()) == sum(want) / (10 * len(sample))
    # a sample id outside [0, n) is reported, not read
    bad = sample.copy()
    bad[7] = n + 5
    est, hits = pg.quality_examination_async(dev(X), dev(cand), 10, bad)
    assert np.isnan(float(est.item())) and int(host(hits)[7]) == -1
    stop = int(0.001 * n * K)
    r = oracle.iter_nsg(X, K, S, 3, 3, stop, k, L, R, 65.0, 3, target=0.995, sample=sample)
    g = pg.iter_nsg(dev(X), K, R, k, L, 65.0, 3, S=S, max_iters=3, seed=3, stop_updates=stop,
                    target=0.995, sample=sample)
    log("rounds", g["rounds"], r["rounds"], "quality", g["quality"], r["quality"])
    assert g["rounds"] == r["rounds"] == 1 and g["quality"] == r["quality"]
    assert np.array_equal(host(g["ids"]), r["ids"])
