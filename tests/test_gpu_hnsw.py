"""Parity of the global HNSW construction (Alg. 7) and its layered search
with the oracle, through the C ABI, on integer data (bit-exact)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def pg():
    from paper_2410_01231_amd import pg as _pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _pg.load_library()
    return _pg


@pytest.mark.parametrize("M", [2, 6, 32, 48])
def test_levels_bit_exact(pg, oracle, datagen, M):
    U = datagen.uniform_open01(300000, seed=M)
    U[:4] = [1.0, 1.0 / M, np.nextafter(1.0 / M, 1.0), 1e-300]
    lev, top = pg.hnsw_levels(dev(U), M)
    ref = oracle.hnsw_levels(U, M)
    assert np.array_equal(host(lev), ref)
    assert top == ref.max()


@pytest.mark.parametrize("n,d,nc,sig,k0,ef,M,alpha,I,S", [
    (1500, 16, 8, 10.0, 12, 16, 6, 65.0, 1, 6),
    (4000, 32, 12, 12.0, 16, 24, 8, 65.0, 2, 8),
])
def test_opt_hnsw_layers_and_search_bit_exact(pg, oracle, datagen, n, d, nc, sig, k0, ef, M, alpha, I, S):
    X, Q = datagen.sift_like(n, 60, d=d, n_clusters=nc, sigma=sig, seed=23)
    U = datagen.uniform_open01(n, seed=3)
    print("opt_hnsw", n, d, M, ef, I, flush=True)
    H = pg.opt_hnsw(dev(X), dev(U), k0, ef, M, alpha, iterations=I, S=S, max_iters=6, seed=2, delta=0.001)
    R = oracle.opt_hnsw(X, U, k0, ef, M, alpha, I, S, 6, 2, 0.001)
    assert H["max_level"] == R["max_level"] >= 2
    assert H["ep"] == R["ep"]
    assert np.array_equal(host(H["levels"]), R["levels"])
    for i, (a, b) in enumerate(zip(H["layers"], R["layers"])):
        assert np.array_equal(host(a["nodes"]), b["nodes"]), i
        assert np.array_equal(host(a["deg"]), b["deg"]), i
        assert np.array_equal(host(a["ids"]), b["ids"]), i
    for k, ef_s in [(10, 24), (1, 1), (10, 64)]:
        ids, d2 = pg.hnsw_search(H, dev(Q), k, ef_s)
        rid, rd2 = oracle.hnsw_search(X, R, Q, k, ef_s)
        assert np.array_equal(host(ids), rid), (k, ef_s)
        assert np.array_equal(host(d2), rd2.astype(np.float32)), (k, ef_s)
