"""Batched builds: several collections in one pg_knn_build_batch call give,
collection by collection, the lists of pg_knn_build on the collection's rows
alone (bit for bit, with each collection's own stop rule and iteration
count), and on integer data the oracle's."""
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


@pytest.mark.parametrize("law,prec", [("int", 0), ("int", 1), ("unit", 0), ("unit", 1), ("unit", 2)])
def test_batch_equals_solo_builds(pg, datagen, oracle, law, prec):
    sizes = [700, 33, 2500, 1200, 65, 4000]
    K, S, T, d = 32, 16, 8, 64
    parts = []
    for i, m in enumerate(sizes):
        if law == "int":
            parts.append(datagen.uniform_int(m, d, seed=100 + i))
        else:
            parts.append(datagen.unit_mixture(m, 0, d=d, n_clusters=8, seed=100 + i)[0])
    X = np.concatenate(parts)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    print("batch", law, prec, sizes, flush=True)
    ids, d2, iters = pg.knn_build_batch(dev(X), off, K, S=S, max_iters=T, seed=5, precision=prec)
    ids, d2 = ids.cpu().numpy(), d2.cpu().numpy()
    for c, m in enumerate(sizes):
        stop = int(0.001 * m * K)
        a, b, st = pg.knn_build(dev(parts[c]), K, S=S, max_iters=T, seed=5, stop_updates=stop, precision=prec)
        assert np.array_equal(ids[off[c]:off[c + 1]], a.cpu().numpy()), c
        assert np.array_equal(d2[off[c]:off[c + 1]].view(np.int32), b.cpu().numpy().view(np.int32)), c
        assert iters[c] == st["iters"], (c, iters[c], st["iters"])
        if law == "int" and c in (1, 3):
            rid, _, _, rst = oracle.nndescent(parts[c], K, S, T, 5, stop_updates=stop)
            assert np.array_equal(ids[off[c]:off[c + 1]], rid)
            assert iters[c] == rst["iters"]


def test_batch_rejects_small_collections(pg, datagen):
    X = dev(datagen.uniform_int(100, 16, seed=1))
    with pytest.raises(pg.PgError) as e:
        pg.knn_build_batch(X, [0, 60, 92, 100], 8, S=4, max_iters=2)
    assert e.value.status == -1 and "collection 2" in str(e.value)
    with pytest.raises(pg.PgError):
        pg.knn_build_batch(X, [0, 60, 90], 8, S=4, max_iters=2)  # does not end at n
