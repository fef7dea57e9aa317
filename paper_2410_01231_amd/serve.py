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

With batch_builds > 1 the dispatcher takes, behind a build of at most
batch_max_rows rows it starts, the next queued builds of the same shape (d,
K, S, R, iteration cap, seed, precision) and size limit that fit, up to
batch_builds of them, and runs their NN-Descent as one batched build
(pg_knn_build_batch: every kernel of an iteration runs once over all the
collections, each with its own stop rule), then refines the collections side
by side.  Each collection's graph is still the one it gets alone.  Small
collections gain (their kernels are too small to fill the GPU on their own);
larger ones already fill it and run alone.
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

    def __init__(self, budget_bytes: int, workers: int = 4, device: int = 0, runner=None, footprint=None,
                 batch_builds: int = 1, batch_max_rows: int = 1 << 15):
        self.budget = int(budget_bytes)
        self.device = device
        self.batch_builds = max(1, int(batch_builds))
        self.batch_max_rows = int(batch_max_rows)
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
        self.batch_log: list[list[str]] = []  # the builds of each batched build
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
                group = [head]
                if head.kind == "build" and self.batch_builds > 1 and self._small(head.payload):
                    group += self._take_batch(head, self._in_use + head.footprint)
                    if len(group) > 1:
                        self.batch_log.append([r.payload.job_id for r in group])
                for r in group:
                    self._in_use += r.footprint
                    self.admission_log.append(f"{r.kind}:{r.payload.job_id}")
                self._running += 1
                if head.kind == "query":
                    self._querying.add(head.payload.job_id)
                self.peak_in_use = max(self.peak_in_use, self._in_use)
            if len(group) > 1:
                self._pool.submit(self._execute_batch, group)
            else:
                self._pool.submit(self._execute, head)

    @staticmethod
    def _shape(job):
        return (job.X.shape[1], job.K, job.S, job.R, job.max_iters, job.seed, job.precision)

    def _small(self, job) -> bool:
        return job.X.shape[0] <= self.batch_max_rows

    def _take_batch(self, head, in_use):
        """The queued builds after `head`, in order, with its shape and that
        fit, up to batch_builds in all (caller holds the lock)."""
        taken, keep = [], collections.deque()
        for r in self._queue:
            if (r.kind == "build" and len(taken) + 1 < self.batch_builds and self._small(r.payload) and
                    self._shape(r.payload) == self._shape(head.payload) and
                    in_use + r.footprint <= self.budget):
                taken.append(r)
                in_use += r.footprint
            else:
                keep.append(r)
        self._queue = keep
        return taken

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

    def _execute_batch(self, group) -> None:
        t0 = time.perf_counter()
        for r in group:
            r.timing.started = t0
        try:
            graphs = self._runner("build_batch", [r.payload for r in group], None)
            errors = [None] * len(group)
        except BaseException as e:  # every build of the batch fails
            graphs, errors = [None] * len(group), [e] * len(group)
        t1 = time.perf_counter()
        with self._cv:
            for r, graph, err in zip(group, graphs, errors):
                jid = r.payload.job_id
                r.timing.finished = t1
                if err is not None:
                    self._state[jid] = "failed"
                    self._fail_queued(jid, f"collection {jid!r} failed to build: {err}")
                elif self._state.get(jid) != "released":
                    self._graphs[jid] = graph
                    self._state[jid] = "ready"
                    self._resident[jid] = r.resident
                    self._in_use += r.resident
                self._in_use -= r.footprint
            self._running -= 1
            self._cv.notify_all()
        for r, graph, err in zip(group, graphs, errors):
            if err is not None:
                r.future.set_exception(err)
            else:
                r.future.set_result((graph, r.timing))

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

    def _gpu_build_batch(self, jobs):
        """NN-Descent of every job in one batched build, then the jobs'
        refinements side by side, each on a stream and context of its own
        (which then serve the collection's queries)."""
        import torch

        from . import pg
        stream = torch.cuda.Stream(self.device)
        dev = f"cuda:{self.device}"
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            ctx = pg.Context(self.device, stream)
            off = np.concatenate([[0], np.cumsum([j.X.shape[0] for j in jobs])]).astype(np.int64)
            Xcat = torch.empty((int(off[-1]), jobs[0].X.shape[1]), dtype=torch.float32, device=dev)
            for c, job in enumerate(jobs):
                Xcat[int(off[c]):int(off[c + 1])].copy_(torch.from_numpy(np.ascontiguousarray(job.X,
                                                                                               dtype=np.float32)))
            j0 = jobs[0]
            ids, d2, iters = pg.knn_build_batch(Xcat, off, j0.K, S=j0.S, max_iters=j0.max_iters, seed=j0.seed,
                                                delta=0.001, precision=j0.precision, ctx=ctx)
            stream.synchronize()

        def refine(c):
            job = jobs[c]
            a, b = int(off[c]), int(off[c + 1])
            qs = torch.cuda.Stream(self.device)
            with torch.cuda.device(self.device), torch.cuda.stream(qs):
                qctx = pg.Context(self.device, qs)
                Xd = Xcat[a:b].clone()
                g = pg.prune(Xd, ids[a:b], job.R, cand_d2=d2[a:b], ctx=qctx)
                x16, exact = pg.half_rows(Xd, ctx=qctx)
                entries = torch.cat([g["ep"], g["roots"]]).contiguous()
                qs.synchronize()
            return {"X": Xd, "ids": g["ids"], "deg": g["deg"], "ep": g["ep"], "roots": g["roots"],
                    "entries": entries, "x16": x16 if exact else None, "ctx": qctx, "stream": qs,
                    "knn_stats": {"iters": iters[c]}}
        with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
            graphs = list(ex.map(refine, range(len(jobs))))
        del Xcat, ids, d2
        return graphs

    def _gpu_run(self, kind, payload, graph):
        import torch

        from . import pg
        if kind == "build_batch":
            return self._gpu_build_batch(payload)
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
