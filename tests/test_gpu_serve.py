"""The serving loop on the GPU: each collection's graph and each query
batch's results are the same when the request runs alone and when it runs in
a mix of overlapping requests admitted against a tight HBM budget."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _jobs(datagen):
    from paper_2410_01231_amd.serve import BuildJob, QueryBatch
    specs = [(2500, 32), (4000, 96), (3000, 32), (6000, 32), (2000, 128), (5000, 64), (1500, 32)]
    jobs, queries = [], []
    for i, (n, d) in enumerate(specs):
        X, Q = datagen.unit_mixture(n, 96, d=d, n_clusters=20, seed=50 + i)
        jobs.append(BuildJob(f"job{i}", X, K=16, R=16, S=8, max_iters=8, seed=3))
        queries.append([QueryBatch(f"job{i}", Q[:40], k=10, L=32), QueryBatch(f"job{i}", Q[40:], k=5, L=48)])
    return jobs, queries


def _host(g):
    return {k: g[k].cpu().numpy() for k in ("ids", "deg", "ep", "roots")}


@pytest.fixture(scope="module")
def alone(datagen):
    from paper_2410_01231_amd.serve import Server
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    jobs, queries = _jobs(datagen)
    # alone: one request at a time
    alone_g, alone_q = {}, {}
    srv = Server(1 << 40, workers=1)
    for j, qs in zip(jobs, queries):
        g, _ = srv.submit_build(j).result(timeout=300)
        alone_g[j.job_id] = _host(g)
        alone_q[j.job_id] = [srv.submit_query(q).result(timeout=300)[0] for q in qs]
        srv.release(j.job_id)
    srv.close()
    return jobs, queries, alone_g, alone_q


@pytest.mark.parametrize("batch", [1, 4])
def test_results_alone_equal_results_in_the_mix(alone, batch):
    # batch > 1: compatible builds run as one batched NN-Descent build
    from paper_2410_01231_amd.serve import Server
    jobs, queries, alone_g, alone_q = alone
    # in the mix: everything submitted at once, four in flight, a budget that
    # holds only a few collections at a time
    fps = sorted((Server._gpu_footprint(None, "build", j)[0] for j in jobs), reverse=True)
    budget = fps[0] + fps[1] + fps[2]
    srv = Server(budget, workers=4, batch_builds=batch)
    fb = [srv.submit_build(j) for j in jobs]
    fq = [[srv.submit_query(q) for q in qs] for qs in queries]
    for j, f, qs in zip(jobs, fb, fq):
        g, timing = f.result(timeout=300)
        got = _host(g)
        for k in got:
            assert np.array_equal(got[k], alone_g[j.job_id][k]), (j.job_id, k)
        for q, want in zip(qs, alone_q[j.job_id]):
            (ids, d2), _ = q.result(timeout=300)
            assert np.array_equal(ids, want[0]) and np.array_equal(d2, want[1]), j.job_id
        srv.release(j.job_id)
    srv.close()
    print(f"[serve] budget {budget} B, peak in use {srv.peak_in_use} B, order {srv.admission_log}, "
          f"batches {srv.batch_log}", flush=True)
    if batch > 1:
        assert srv.batch_log  # some builds ran batched
    assert srv.peak_in_use <= budget
