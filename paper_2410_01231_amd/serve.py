"""Serving loop: build jobs and k-ANN query batches on one GPU, admitted by
HBM footprint, overlapped on the device.

Every admitted request runs on a worker thread with its own HIP stream and
library context, so the build kernels of different collections and their
query batches overlap on the GPU (the library's calls release the GIL while
they wait on their own stream).  Admission runs against an HBM ledger: a
request starts once the footprint it declares fits beside the ones running
and the graphs kept resident; builds start in arrival order, and a query
whose collection is built may start ahead of builds still waiting for
memory.  A request larger than the whole budget is rejected.  A build keeps
its collection's rows and graph resident (counted in the ledger) until
release().  Queries of one collection share its library context, so they
run one at a time: a query is not admitted while another query of the same
collection runs, and holds no slot or memory while it waits.  A query for a
collection whose build failed, that was released or that was never
submitted fails at once; queries still queued when their build fails or
their collection is released fail then, and close() fails whatever can no
longer run.  Results do not depend on what else runs: every kernel of the
library is deterministic, so a collection's graph and a query's results are
the same alone and in the mix.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class BuildJob:
    """One collection to index: rows X (n x d float32, host), kNN width K,
    degree bound R, NN-Descent sample S and iteration cap."""
    job_id: str
    X: np.ndarray
    K: int = 32
    R: int = 32
    S: int = 16
    max_iters: int = 12
    seed: int = 1
    precision: int = 0


@dataclass
class QueryBatch:
    job_id: str
    Q: np.ndarray
    k: int = 10
    L: int = 64


@dataclass
class Timing:
    submitted: float = 0.0
    started: float = 0.0
    finished: float = 0.0

    @property
    def latency(self) -> float:
        return self.finished - self.submitted

    @property
    def service(self) -> float:
        return self.finished - self.started


class AdmissionError(RuntimeError):
    pass


class CollectionError(RuntimeError):
    """A query names a collection with no graph to answer it: its build
    failed, it was released, or it was never submitted."""


@dataclass
class _Request:
    kind: str                # "build" or "query"
    payload: object
    footprint: int           # bytes held while it runs
    resident: int            # bytes kept after a build finishes (its graph)
    future: Future
    timing: Timing = field(default_factory=Timing)


class Server:
    """Admission against an HBM budget, `workers` requests in flight.

    runner(kind, payload, state) -> result runs one request; the default runs
    it on the GPU through the library.  footprint(kind, payload) -> (bytes
    while running, bytes kept after) sizes it; the default asks the library
    for its workspace sizes.  Both can be replaced (tests drive the ledger
    with fakes)."""

    def __init__(self, budget_bytes: int, workers: int = 4, device: int = 0, runner=None, footprint=None):
        self.budget = int(budget_bytes)
        self.device = device
        self._runner = runner or self._gpu_run
        self._footprint = footprint or self._gpu_footprint
        self._pool = ThreadPoolExecutor(max_workers=workers)
        self._slots = workers
        self._queue: collections.deque[_Request] = collections.deque()
        self._cv = threading.Condition()
        self._in_use = 0          # bytes of running requests plus resident graphs
        self._running = 0
        self._resident: dict[str, int] = {}
        self._graphs: dict[str, object] = {}
        # collection state: "building" (build submitted, no graph yet), "ready",
        # "failed" or "released"; absent = never submitted
        self._state: dict[str, str] = {}
        self._querying: set[str] = set()   # collections with a query running
        self.peak_in_use = 0
        self.admission_log: list[str] = []
        self._closed = False
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        self._dispatcher.start()

    # ------------------------------------------------------------------ API
    def submit_build(self, job: BuildJob) -> Future:
        fp, res = self._footprint("build", job)
        return self._enqueue("build", job, fp, res)

    def submit_query(self, batch: QueryBatch) -> Future:
        fp, _ = self._footprint("query", batch)
        return self._enqueue("query", batch, fp, 0)

    def release(self, job_id: str) -> None:
        """Drop a collection's resident graph and give its bytes back; its
        queued queries fail.  A collection still building is dropped when its
        build ends."""
        with self._cv:
            self._graphs.pop(job_id, None)
            self._in_use -= self._resident.pop(job_id, 0)
            if job_id in self._state:
                self._state[job_id] = "released"
            self._fail_queued(job_id, f"collection {job_id!r} was released")
            self._cv.notify_all()

    def close(self) -> None:
        """Stop taking requests, run what can still run, fail the rest."""
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        self._dispatcher.join()
        self._pool.shutdown(wait=True)

    # ------------------------------------------------------------ internals
    def _enqueue(self, kind, payload, fp, res) -> Future:
        fut: Future = Future()
        req = _Request(kind, payload, int(fp), int(res), fut)
        req.timing.submitted = time.perf_counter()
        if req.footprint > self.budget:
            fut.set_exception(AdmissionError(
                f"{kind} request needs {req.footprint} bytes, more than the budget of {self.budget}"))
            return fut
        with self._cv:
            if self._closed:
                fut.set_exception(AdmissionError("the server is closed"))
                return fut
            job_id = payload.job_id
            if kind == "build":
                if self._state.get(job_id) in ("building", "ready"):
                    fut.set_exception(AdmissionError(f"collection {job_id!r} is already built or building"))
                    return fut
                self._state[job_id] = "building"
            else:
                st = self._state.get(job_id)
                if st not in ("building", "ready"):
                    why = "was never submitted" if st is None else ("failed to build" if st == "failed"
                                                                    else "was released")
                    fut.set_exception(CollectionError(f"collection {job_id!r} {why}"))
                    return fut
            self._queue.append(req)
            self._cv.notify_all()
        return fut

    def _fail_queued(self, job_id, why) -> None:
        """Fail the queued queries of a collection (caller holds the lock)."""
        keep = collections.deque()
        for r in self._queue:
            if r.kind == "query" and r.payload.job_id == job_id:
                r.timing.finished = time.perf_counter()
                r.future.set_exception(CollectionError(why))
            else:
                keep.append(r)
        self._queue = keep

    def _runnable(self, r: _Request) -> bool:
        """A queued request can still start some day."""
        return r.kind == "build" or self._state.get(r.payload.job_id) in ("building", "ready")

    def _dispatch(self) -> None:
        while True:
            with self._cv:
                while True:
                    if self._closed:
                        dead = [r for r in self._queue if not self._runnable(r)]
                        for r in dead:
                            self._fail_queued(r.payload.job_id, f"collection {r.payload.job_id!r} has no graph")
                    if self._closed and not self._queue and self._running == 0:
                        return
                    i = self._pick() if self._running < self._slots else None
                    if i is not None:
                        head = self._queue[i]
                        del self._queue[i]
                        break
                    self._cv.wait(timeout=0.05)
                self._in_use += head.footprint
                self._running += 1
                if head.kind == "query":
                    self._querying.add(head.payload.job_id)
                self.peak_in_use = max(self.peak_in_use, self._in_use)
                name = head.payload.job_id
                self.admission_log.append(f"{head.kind}:{name}")
            self._pool.submit(self._execute, head)

    def _pick(self):
        """Index of the next request to start: builds in arrival order (a build
        that does not fit holds back the later ones), queries as soon as their
        collection is built, no other query of it runs and they fit, ahead of
        waiting builds."""
        build_blocked = False
        for i, r in enumerate(self._queue):
            fits = self._in_use + r.footprint <= self.budget
            if r.kind == "build":
                if build_blocked:
                    continue
                if fits:
                    return i
                build_blocked = True
            elif fits and self._ready(r):
                return i
        return None

    def _ready(self, req: _Request) -> bool:
        # a query waits for its collection's graph and for the collection's
        # running query (they share one library context)
        return req.kind != "query" or (req.payload.job_id in self._graphs and
                                       req.payload.job_id not in self._querying)

    def _execute(self, req: _Request) -> None:
        req.timing.started = time.perf_counter()
        try:
            if req.kind == "build":
                graph = self._runner("build", req.payload, None)
                with self._cv:
                    # a collection released while it was building keeps nothing
                    if self._state.get(req.payload.job_id) != "released":
                        self._graphs[req.payload.job_id] = graph
                        self._state[req.payload.job_id] = "ready"
                        self._resident[req.payload.job_id] = req.resident
                        self._in_use += req.resident
                result = graph
            else:
                with self._cv:
                    graph = self._graphs.get(req.payload.job_id)
                if graph is None:
                    raise CollectionError(f"collection {req.payload.job_id!r} was released")
                result = self._runner("query", req.payload, graph)
            req.timing.finished = time.perf_counter()
            req.future.set_result((result, req.timing))
        except BaseException as e:  # the request fails, the server goes on
            req.timing.finished = time.perf_counter()
            if req.kind == "build":
                with self._cv:
                    self._state[req.payload.job_id] = "failed"
                    self._fail_queued(req.payload.job_id,
                                      f"collection {req.payload.job_id!r} failed to build: {e}")
            req.future.set_exception(e)
        finally:
            with self._cv:
                self._in_use -= req.footprint
                self._running -= 1
                if req.kind == "query":
                    self._querying.discard(req.payload.job_id)
                self._cv.notify_all()

    # --------------------------------------------------------------- GPU side
    def _gpu_footprint(self, kind, payload):
        from . import pg
        if kind == "query":
            nq, d = payload.Q.shape
            return nq * d * 4 + nq * payload.k * 8 + (1 << 20), 0
        n, d = payload.X.shape
        job = payload
        rows = n * d * 4 + n * ((d + 7) // 8 * 8) * 2          # X and its FP16 copy
        graph = n * job.R * 8 + n * 4 * 3                        # ids, d2, deg, roots
        lists = n * job.K * 8
        knn_ws = pg.knn_workspace_bytes(n, d, job.K, job.S, job.max_iters, job.precision)
        prune_ws = pg.prune_workspace_bytes(n, d, job.K, job.R)
        return rows + graph + lists + knn_ws + prune_ws, rows + graph

    def _gpu_run(self, kind, payload, graph):
        import torch

        from . import pg
        if kind == "build":
            job = payload
            stream = torch.cuda.Stream(self.device)
            with torch.cuda.device(self.device), torch.cuda.stream(stream):
                ctx = pg.Context(self.device, stream)
                Xd = torch.from_numpy(np.ascontiguousarray(job.X, dtype=np.float32)).to(
                    f"cuda:{self.device}")
                ids, d2, st = pg.knn_build(Xd, job.K, S=job.S, max_iters=job.max_iters, seed=job.seed,
                                           delta=0.001, precision=job.precision, ctx=ctx)
                g = pg.prune(Xd, ids, job.R, cand_d2=d2, ctx=ctx)
                x16, exact = pg.half_rows(Xd, ctx=ctx)
                entries = torch.cat([g["ep"], g["roots"]]).contiguous()
                del ids, d2
                stream.synchronize()
            return {"X": Xd, "ids": g["ids"], "deg": g["deg"], "ep": g["ep"], "roots": g["roots"],
                    "entries": entries, "x16": x16 if exact else None, "ctx": ctx, "stream": stream,
                    "knn_stats": st}
        batch = payload
        stream = graph["stream"]
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            Qd = torch.from_numpy(np.ascontiguousarray(batch.Q, dtype=np.float32)).to(f"cuda:{self.device}")
            ids, d2 = pg.search(graph["X"], graph["ids"], graph["deg"], Qd, graph["entries"], batch.k, batch.L,
                                x16=graph["x16"], ctx=graph["ctx"])
            out = (ids.cpu().numpy(), d2.cpu().numpy())
            stream.synchronize()
        return out


def percentiles(values, ps=(50, 99)):
    v = np.asarray(values, dtype=np.float64)
    return {f"p{p}": float(np.percentile(v, p)) if v.size else None for p in ps}
