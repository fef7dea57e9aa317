"""pg_knn_build_noalloc (workspace in the library's static device scratch)
against pg_knn_build with a caller workspace: identical lists, distances and
counters on two calls in a row, the second one smaller (the scratch keeps the
first call's contents, so whatever must start at zero has to be cleared by the
call itself), on float data (FP32 direct form and FP16 mixed precision) and on
integer data, where the lists must also equal the oracle's bit for bit.  A
build larger than the scratch is refused before any work is enqueued."""
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


def _same(pg, X, K, S, T, prec, seed):
    stop = int(0.001 * X.shape[0] * K)
    print("noalloc case", X.shape, K, S, T, prec, seed, flush=True)
    a_ids, a_d2, a_st = pg.knn_build_noalloc(X, K, S=S, max_iters=T, seed=seed, stop_updates=stop,
                                             precision=prec)
    b_ids, b_d2, b_st = pg.knn_build(X, K, S=S, max_iters=T, seed=seed, stop_updates=stop, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(a_ids, b_ids)
    assert torch.equal(a_d2.view(torch.int32), b_d2.view(torch.int32))
    # the counters that the result defines (the spill, retry and emission
    # counts depend on the order of the proposal atomics, run to run)
    for key in ("iters", "updates", "pairs", "members", "join_path"):
        assert a_st[key] == b_st[key], key
    return a_ids, a_st


def test_noalloc_equals_workspace_build_twice_then_smaller(pg, datagen, oracle):
    # first call: float data, FP32 direct form, the larger input
    X1, _ = datagen.gist_like(6000, 0, d=64, seed=3)
    _same(pg, dev(X1), 32, 16, 6, pg.FP32_VALU, 1)
    # second call, smaller, FP16 mixed precision on the same float law
    X2, _ = datagen.gist_like(2500, 0, d=96, seed=5)
    _, st2 = _same(pg, dev(X2), 24, 12, 5, pg.FP16, 2)
    assert st2["join_path"] == "fp16-mixed"
    # third call, smaller again: integer data, MFMA path, equal to the oracle
    X3 = datagen.uniform_int(1200, 32, seed=7)
    ids3, st3 = _same(pg, dev(X3), 16, 8, 5, pg.FP32, 4)
    assert st3["join_path"] == "fp32-mfma"
    rid, _, _, _ = oracle.nndescent(X3, 16, 8, 5, 4, stop_updates=int(0.001 * 1200 * 16))
    assert np.array_equal(ids3.cpu().numpy(), rid)


def test_noalloc_refuses_builds_beyond_the_scratch(pg):
    n, d, K = 60_000, 128, 32
    assert pg.knn_workspace_bytes(n, d, K, 16) > pg.NOALLOC_WS_BYTES
    X = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    with pytest.raises(pg.PgError) as e:
        pg.knn_build_noalloc(X, K, S=16, max_iters=2)
    assert e.value.status == -2 and "static scratch" in str(e.value)
    # a refused call leaves the scratch usable
    Xs = torch.from_numpy(np.arange(64 * 8, dtype=np.float32).reshape(64, 8) % 17).cuda()
    _same(pg, Xs, 8, 4, 3, pg.FP32_VALU, 0)
