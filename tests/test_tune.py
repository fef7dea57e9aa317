"""The autotuner's host logic (shape keys, the fastest setting, the JSON
cache) on the CPU, and on the GPU that tuned builds give the default build's
lists and that a cached shape runs no probes."""
import json

import numpy as np
import pytest


def test_shape_key_rounds_rows_up_to_a_power_of_two():
    from paper_2410_01231_amd.tune import shape_key
    assert shape_key(1000, 128, 32, 16, "fp32-valu") == "n1024-d128-K32-S16-fp32-valu"
    assert shape_key(1024, 128, 32, 16, "fp32-valu") == "n1024-d128-K32-S16-fp32-valu"
    assert shape_key(1025, 96, 64, 32, "fp16-mixed") == "n2048-d96-K64-S32-fp16-mixed"


def test_choose_takes_the_fastest_and_the_earlier_on_ties():
    from paper_2410_01231_amd.tune import choose
    t = [(5.0, {"a": 1}), (3.0, {"a": 2}), (3.0, {"a": 3}), (9.0, {"a": 4})]
    assert choose(t) == {"a": 2, "ms": 3.0}


def test_candidates_cover_both_precisions():
    from paper_2410_01231_amd import pg
    from paper_2410_01231_amd.tune import candidates
    c = candidates(960)
    assert {s["precision"] for s in c} == {pg.FP32, pg.FP16}
    assert {s["precision"] for s in candidates(96)} == {pg.FP32, pg.BF16}
    assert len(c) == len({json.dumps(s, sort_keys=True) for s in c})


@pytest.mark.gpu
def test_tuned_build_equals_default_build_and_caches(tmp_path, datagen):
    import torch
    from paper_2410_01231_amd import pg, tune
    X, _ = datagen.unit_mixture(3000, 0, d=96, n_clusters=10, seed=3)
    Xd = torch.from_numpy(X).cuda()
    path = str(tmp_path / "tune.json")
    calls = []

    def timer(fn):
        calls.append(1)
        fn()
        return float(len(calls) % 5)   # any timings: the lists must not depend on them
    kn = tune.tune_knn(Xd, 24, S=12, seed=2, cache_path=path, timer=timer)
    assert len(calls) == len(tune.candidates(96))   # every setting fits beside this small set
    table = json.load(open(path))
    assert len(table) == 1
    a = pg.knn_build(Xd, 24, S=12, max_iters=6, seed=2, **kn)
    b = pg.knn_build(Xd, 24, S=12, max_iters=6, seed=2)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # the same shape again: no probes (from memory, then from the file alone)
    tune.tune_knn(Xd, 24, S=12, seed=2, cache_path=path, timer=timer)
    tune._cache.clear()
    assert tune.tune_knn(Xd, 24, S=12, seed=2, cache_path=path, timer=timer) == kn
    assert len(calls) == len(tune.candidates(96))
