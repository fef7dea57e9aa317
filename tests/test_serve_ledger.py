"""Admission of the serving loop, driven on the CPU with a fake runner and
fake footprints: FIFO order against the HBM budget, rejection of requests
larger than the budget, resident graphs held until release, queries waiting
for their collection, and a failing request leaving the server running."""
import threading
import time

import numpy as np
import pytest

from paper_2410_01231_amd.serve import AdmissionError, BuildJob, CollectionError, QueryBatch, Server


class Fake:
    def __init__(self, sizes):
        self.sizes = sizes                  # job_id -> (running bytes, resident bytes)
        self.gates = {k: threading.Event() for k in sizes}
        self.started = []
        self.lock = threading.Lock()

    def footprint(self, kind, payload):
        if kind == "query":
            return 1, 0
        return self.sizes[payload.job_id]

    def runner(self, kind, payload, graph):
        with self.lock:
            self.started.append(f"{kind}:{payload.job_id}")
        if kind == "build":
            if payload.job_id == "bad":
                raise ValueError("broken job")
            assert self.gates[payload.job_id].wait(5.0)
            return {"graph_of": payload.job_id}
        return ("answer", payload.job_id, graph["graph_of"])


def job(name):
    return BuildJob(name, np.zeros((4, 4), np.float32))


def wait_until(cond, timeout=5.0):
    t0 = time.time()
    while not cond():
        assert time.time() - t0 < timeout, "timed out"
        time.sleep(0.005)


def test_fifo_admission_and_rejection():
    f = Fake({"A": (60, 0), "B": (50, 0), "C": (30, 0), "D": (120, 0)})
    srv = Server(100, workers=4, runner=f.runner, footprint=f.footprint)
    fa, fb, fc = srv.submit_build(job("A")), srv.submit_build(job("B")), srv.submit_build(job("C"))
    fd = srv.submit_build(job("D"))
    with pytest.raises(AdmissionError):
        fd.result(timeout=1)
    wait_until(lambda: f.started == ["build:A"])
    time.sleep(0.1)
    assert f.started == ["build:A"]          # B does not fit beside A, C waits behind B
    f.gates["A"].set()
    fa.result(timeout=5)
    wait_until(lambda: len(f.started) == 3)
    assert f.started[1:] == ["build:B", "build:C"]   # 50 + 30 fit together
    f.gates["B"].set()
    f.gates["C"].set()
    fb.result(timeout=5)
    fc.result(timeout=5)
    srv.close()
    assert srv.admission_log == ["build:A", "build:B", "build:C"]
    assert srv.peak_in_use <= 100


def test_resident_graph_held_until_release_and_queries_wait():
    f = Fake({"A": (60, 40), "B": (70, 10)})
    srv = Server(100, workers=4, runner=f.runner, footprint=f.footprint)
    fa = srv.submit_build(job("A"))
    fq = srv.submit_query(QueryBatch("A", np.zeros((2, 4), np.float32)))
    time.sleep(0.1)
    assert f.started == ["build:A"]          # the query waits for A's graph
    f.gates["A"].set()
    (graph, _), (ans, _) = fa.result(timeout=5), fq.result(timeout=5)
    assert ans == ("answer", "A", "A")
    fb = srv.submit_build(job("B"))
    time.sleep(0.15)
    assert "build:B" not in f.started        # A's resident 40 + 70 > 100
    srv.release("A")
    wait_until(lambda: "build:B" in f.started)
    f.gates["B"].set()
    fb.result(timeout=5)
    srv.close()


def test_failing_request_does_not_stop_the_server():
    f = Fake({"bad": (10, 0), "A": (10, 0)})
    srv = Server(100, workers=2, runner=f.runner, footprint=f.footprint)
    fbad = srv.submit_build(job("bad"))
    with pytest.raises(ValueError):
        fbad.result(timeout=5)
    f.gates["A"].set()
    (g, timing) = srv.submit_build(job("A")).result(timeout=5)
    assert g == {"graph_of": "A"} and timing.latency >= timing.service >= 0
    srv.close()


def test_query_after_failed_build_fails():
    f = Fake({"bad": (10, 0)})
    srv = Server(100, workers=2, runner=f.runner, footprint=f.footprint)
    fbad = srv.submit_build(job("bad"))
    fq = srv.submit_query(QueryBatch("bad", np.zeros((2, 4), np.float32)))   # queued before the failure
    with pytest.raises(ValueError):
        fbad.result(timeout=5)
    with pytest.raises(CollectionError):
        fq.result(timeout=5)
    with pytest.raises(CollectionError):                                      # submitted after it
        srv.submit_query(QueryBatch("bad", np.zeros((2, 4), np.float32))).result(timeout=5)
    srv.close()


def test_query_for_unknown_or_released_collection_fails():
    f = Fake({"A": (10, 5)})
    srv = Server(100, workers=2, runner=f.runner, footprint=f.footprint)
    with pytest.raises(CollectionError, match="never submitted"):
        srv.submit_query(QueryBatch("nope", np.zeros((1, 4), np.float32))).result(timeout=5)
    fa = srv.submit_build(job("A"))
    fq = srv.submit_query(QueryBatch("A", np.zeros((1, 4), np.float32)))
    srv.release("A")                                                          # before the graph exists
    with pytest.raises(CollectionError, match="released"):
        fq.result(timeout=5)
    f.gates["A"].set()
    fa.result(timeout=5)
    srv.release("A")
    with pytest.raises(CollectionError, match="released"):
        srv.submit_query(QueryBatch("A", np.zeros((1, 4), np.float32))).result(timeout=5)
    srv.close()
    assert srv._in_use == 0


def test_close_with_pending_queries_returns():
    f = Fake({"A": (10, 0), "B": (10, 0)})
    srv = Server(100, workers=2, runner=f.runner, footprint=f.footprint)
    fa = srv.submit_build(job("A"))
    qs = [srv.submit_query(QueryBatch("A", np.zeros((1, 4), np.float32))) for _ in range(3)]
    closer = threading.Thread(target=srv.close)
    closer.start()
    time.sleep(0.1)
    f.gates["A"].set()                         # the build and its queries can still run
    closer.join(timeout=5)
    assert not closer.is_alive()
    fa.result(timeout=1)
    for q in qs:
        assert q.result(timeout=1)[0] == ("answer", "A", "A")
    with pytest.raises(AdmissionError):
        srv.submit_build(job("B")).result(timeout=1)


def test_queries_of_one_collection_wait_outside_admission():
    # a second query of a collection whose query runs takes no slot: a query
    # of another collection starts beside it
    started = threading.Event()
    release_q = threading.Event()
    order = []

    def runner(kind, payload, graph):
        if kind == "build":
            return {"graph_of": payload.job_id}
        order.append(payload.job_id)
        if payload.job_id == "A" and not started.is_set():
            started.set()
            assert release_q.wait(5)
        return payload.job_id

    srv = Server(100, workers=2, runner=runner, footprint=lambda k, p: (1, 0))
    srv.submit_build(job("A")).result(timeout=5)
    srv.submit_build(job("B")).result(timeout=5)
    q1 = srv.submit_query(QueryBatch("A", np.zeros((1, 4), np.float32)))
    assert started.wait(5)
    q2 = srv.submit_query(QueryBatch("A", np.zeros((1, 4), np.float32)))
    q3 = srv.submit_query(QueryBatch("B", np.zeros((1, 4), np.float32)))
    assert q3.result(timeout=5)[0] == "B"      # B ran while A's second query waited
    assert not q2.done()
    release_q.set()
    assert q1.result(timeout=5)[0] == "A" and q2.result(timeout=5)[0] == "A"
    assert order == ["A", "B", "A"]
    srv.close()


def test_compatible_builds_are_batched_within_the_budget():
    # batch_builds = 3: behind the build it starts, the dispatcher takes the
    # next queued builds of the same shape that fit, up to three in all; a
    # build of another shape and one that does not fit wait for later
    batches = []

    def runner(kind, payload, graph):
        if kind == "build_batch":
            batches.append([j.job_id for j in payload])
            return [{"graph_of": j.job_id} for j in payload]
        if kind == "build":
            batches.append([payload.job_id])
            return {"graph_of": payload.job_id}
        return ("answer", payload.job_id, graph["graph_of"])

    sizes = {"A": 10, "B": 10, "W": 10, "C": 10, "D": 90, "E": 10, "F": 10}

    def footprint(kind, payload):
        return (1, 0) if kind == "query" else (sizes[payload.job_id], 2)

    srv = Server(100, workers=1, runner=runner, footprint=footprint, batch_builds=3)
    wide = BuildJob("W", np.zeros((4, 8), np.float32))
    futs = [srv.submit_build(job(x)) for x in "AB"] + [srv.submit_build(wide)] + \
        [srv.submit_build(job(x)) for x in "CDEF"]
    q = srv.submit_query(QueryBatch("C", np.zeros((1, 4), np.float32)))
    for f, name in zip(futs, "ABWCDEF"):
        g, _ = f.result(timeout=5)
        assert g == {"graph_of": name}
    assert q.result(timeout=5)[0] == ("answer", "C", "C")
    srv.close()
    # every build ran exactly once; batches hold one shape and fit the budget
    assert sorted(sum(batches, [])) == sorted("ABWCDEF")
    assert batches[0] == ["A", "B", "C"]
    for b in batches:
        assert len(b) <= 3
        assert len({("W" in b and x == "W") or x == "W" for x in b}) == 1
        assert sum(sizes[x] for x in b) <= 100
    assert srv.peak_in_use <= 100
