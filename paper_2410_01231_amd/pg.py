"""Thin Python binding of the C ABI in include/pg.h (libpg.so, gfx950 HIP kernels).

Argument marshalling only: every step of the build and search runs in the
library's kernels.  torch supplies device memory and the current HIP stream.
The library must be built (``paper_2410_01231_amd.build.build()``); there is no
fallback of any kind, so importing a function without the library raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, \
    c_uint32, c_uint64, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpg.so")

STAGE_PRUNE, STAGE_REVERSE, STAGE_CONNECT = 1, 2, 4
STAGES_ALL = STAGE_PRUNE | STAGE_REVERSE | STAGE_CONNECT
FP32, FP16, BF16, FP32_VALU = 0, 1, 2, 3
JOIN_PATHS = {0: "fp32-valu", 1: "fp32-mfma", 2: "fp16-mfma", 3: "bf16-mfma", 4: "fp16-mixed",
              5: "bf16-mixed"}


class PgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pg status {status}: {msg}")
        self.status = status


class KnnParams(ctypes.Structure):
    _fields_ = [("K", c_int32), ("S", c_int32), ("max_iters", c_int32), ("exact", c_int32),
                ("stop_updates", c_int64), ("seed", c_uint64), ("precision", c_int32),
                ("margin_rel", c_float), ("bucket_cap", c_int32), ("chunks", c_int32)]


class KnnStats(ctypes.Structure):
    _fields_ = [("iters_run", c_int32), ("join_path", c_int32), ("updates", c_int64 * 64),
                ("pairs", c_int64 * 64), ("proposals", c_int64 * 64), ("retries", c_int64),
                ("spilled", c_int64), ("rechecked", c_int64 * 64), ("members", c_int64 * 64)]


class PruneParams(ctypes.Structure):
    _fields_ = [("R", c_int32), ("alpha_deg", c_float), ("stages", c_uint32),
                ("strict_ties", c_int32), ("pair_d2", c_void_p), ("precision", c_int32),
                ("k2p_prev_ids", c_void_p), ("k2p_prev_deg", c_void_p), ("k2p_prev_R", c_int32),
                ("k2p_counts", c_void_p), ("prune_ids_out", c_void_p), ("prune_deg_out", c_void_p)]


class SearchParams(ctypes.Structure):
    _fields_ = [("k", c_int32), ("L", c_int32), ("n_entry", c_int32), ("entry_ids", c_void_p),
                ("query_entry", c_void_p), ("exclude", c_void_p), ("record_ids", c_void_p),
                ("record_d2", c_void_p), ("record_L", c_int32), ("pool_ids", c_void_p),
                ("pool_d2", c_void_p), ("counts", c_void_p), ("x16", c_void_p)]


EXPORTS = ["pg_version", "pg_last_error", "pg_ctx_create", "pg_ctx_destroy", "pg_ctx_set_timing",
           "pg_ctx_kernel_time", "pg_ctx_reset_timing", "pg_knn_build_workspace", "pg_knn_build",
           "pg_exact_knn", "pg_prune_workspace", "pg_prune", "pg_search", "pg_hnsw_levels",
           "pg_half_rows", "pg_knn_build_noalloc", "pg_quality_examination", "pg_knn_build_batch_workspace",
           "pg_knn_build_batch"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpg.so and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2410_01231_amd.build.build()")
    lib = ctypes.CDLL(path)
    P = c_void_p
    lib.pg_version.restype = c_int
    lib.pg_last_error.restype = c_char_p
    lib.pg_ctx_create.argtypes = [c_int, P, POINTER(c_void_p)]
    lib.pg_ctx_destroy.argtypes = [P]
    lib.pg_ctx_set_timing.argtypes = [P, c_int]
    lib.pg_ctx_reset_timing.argtypes = [P]
    lib.pg_ctx_kernel_time.argtypes = [P, c_char_p, POINTER(c_double), POINTER(c_int64),
                                       POINTER(c_double)]
    lib.pg_knn_build_workspace.argtypes = [POINTER(KnnParams), c_int64, c_int32, POINTER(c_size_t)]
    lib.pg_knn_build.argtypes = [P, P, c_int64, c_int32, c_int64, POINTER(KnnParams), P, c_size_t,
                                 P, P, POINTER(KnnStats)]
    lib.pg_knn_build_noalloc.argtypes = [P, P, c_int64, c_int32, c_int64, POINTER(KnnParams), P, P,
                                         POINTER(KnnStats)]
    lib.pg_knn_build_batch_workspace.argtypes = [POINTER(KnnParams), c_int64, c_int32, c_int32, POINTER(c_size_t)]
    lib.pg_knn_build_batch.argtypes = [P, P, c_int64, c_int32, c_int64, P, c_int32, P, POINTER(KnnParams), P,
                                       c_size_t, P, P, P]
    lib.pg_quality_examination.argtypes = [P, P, c_int64, c_int32, c_int64, P, c_int32, c_int32, P, c_int64,
                                           P, P, P, P]
    lib.pg_exact_knn.argtypes = [P, P, c_int64, c_int32, c_int64, P, c_int64, c_int64, P, c_int32,
                                 P, P]
    lib.pg_prune_workspace.argtypes = [POINTER(PruneParams), c_int64, c_int32, c_int32,
                                       POINTER(c_size_t)]
    lib.pg_prune.argtypes = [P, P, c_int64, c_int32, c_int64, P, P, c_int32, POINTER(PruneParams), P,
                             c_size_t, P, P, P, P, P, POINTER(c_int32)]
    lib.pg_search.argtypes = [P, P, c_int64, c_int32, c_int64, P, c_int32, P, P, c_int64, c_int64,
                              POINTER(SearchParams), P, P]
    lib.pg_hnsw_levels.argtypes = [P, P, c_int64, c_int32, P, P]
    lib.pg_half_rows.argtypes = [P, P, c_int64, c_int32, c_int64, P, P]
    for name in EXPORTS:
        f = getattr(lib, name)
        if name not in ("pg_version", "pg_last_error"):
            f.restype = c_int
    _lib = lib
    return lib


def _check(status, what):
    if status != 0:
        msg = load_library().pg_last_error().decode()
        raise PgError(status, f"{what}: {msg}")


class Context:
    """A pg_ctx bound to a device and a HIP stream (torch's current stream by default)."""

    def __init__(self, device=None, stream=None):
        lib = load_library()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = c_void_p()
        _check(lib.pg_ctx_create(dev.index, c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "pg_ctx_create")
        self.handle = h

    def set_timing(self, enable: bool):
        _check(load_library().pg_ctx_set_timing(self.handle, int(bool(enable))), "set_timing")

    def reset_timing(self):
        _check(load_library().pg_ctx_reset_timing(self.handle), "reset_timing")

    def kernel_time(self, name: str):
        """(total_ms, launches, work) of the named kernel since the last reset."""
        ms, cnt, work = c_double(), c_int64(), c_double()
        _check(load_library().pg_ctx_kernel_time(self.handle, name.encode(), ctypes.byref(ms),
                                                 ctypes.byref(cnt), ctypes.byref(work)),
               "kernel_time")
        return ms.value, cnt.value, work.value

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.pg_ctx_destroy(self.handle)
        except Exception:
            pass


_contexts = {}


def context(device=None) -> Context:
    """The cached context for the device's current stream."""
    dev = torch.cuda.current_device() if device is None else device
    s = torch.cuda.current_stream(dev)
    key = (dev, s.cuda_stream)
    if key not in _contexts:
        _contexts[key] = Context(dev, s)
    return _contexts[key]


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _dev_f32(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 2):
        raise TypeError(f"{name} must be a 2-D float32 device tensor")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit stride along its rows")
    return t


def _dev_i32(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32):
        raise TypeError(f"{name} must be an int32 device tensor")
    return t.contiguous()


def knn_workspace_bytes(n, d, K, S=None, max_iters=12, precision=FP32, bucket_cap=0):
    """Workspace bytes pg_knn_build needs for n rows of d dimensions."""
    lib = load_library()
    S = (K + 1) // 2 if S is None else S
    p = KnnParams(K=K, S=S, max_iters=max_iters, precision=precision, bucket_cap=bucket_cap)
    ws = c_size_t()
    _check(lib.pg_knn_build_workspace(ctypes.byref(p), n, d, ctypes.byref(ws)), "workspace")
    return int(ws.value)


def prune_workspace_bytes(n, d, C, R, alpha_deg=60.0):
    """Workspace bytes pg_prune needs for n candidate lists of C ids."""
    lib = load_library()
    p = PruneParams(R=R, alpha_deg=float(alpha_deg), stages=STAGES_ALL)
    ws = c_size_t()
    _check(lib.pg_prune_workspace(ctypes.byref(p), n, d, C, ctypes.byref(ws)), "workspace")
    return int(ws.value)


def knn_build(X, K, S=None, max_iters=12, seed=0, stop_updates=None, delta=0.001, exact=False,
              bucket_cap=0, chunks=0, precision=FP32, margin_rel=0.0, ctx=None):
    """NN-Descent kNN lists of the rows of X: returns (ids, d2, stats dict)."""
    lib = load_library()
    X = _dev_f32(X, "X")
    n, d = X.shape
    S = (K + 1) // 2 if S is None else S
    if stop_updates is None:
        stop_updates = int(delta * n * K)
    p = KnnParams(K=K, S=S, max_iters=max_iters, exact=int(bool(exact)), stop_updates=stop_updates,
                  seed=seed & (2**64 - 1), precision=precision, margin_rel=float(margin_rel),
                  bucket_cap=bucket_cap,
                  chunks=chunks)
    ws_bytes = c_size_t()
    _check(lib.pg_knn_build_workspace(ctypes.byref(p), n, d, ctypes.byref(ws_bytes)), "workspace")
    ws = torch.empty(max(ws_bytes.value, 1), dtype=torch.uint8, device=X.device)
    ids = torch.empty((n, K), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, K), dtype=torch.float32, device=X.device)
    st = KnnStats()
    ctx = ctx or context(X.device.index)
    _check(lib.pg_knn_build(ctx.handle, _ptr(X), n, d, X.stride(0), ctypes.byref(p), _ptr(ws),
                            ws_bytes.value, _ptr(ids), _ptr(d2), ctypes.byref(st)), "pg_knn_build")
    it = st.iters_run
    stats = {"iters": it, "updates": list(st.updates[:it]), "pairs": list(st.pairs[:it]),
             "proposals": list(st.proposals[:it]), "rechecked": list(st.rechecked[:it]),
             "members": list(st.members[:it]),
             "retries": st.retries,
             "spilled": st.spilled, "join_path": JOIN_PATHS.get(st.join_path, st.join_path)}
    return ids, d2, stats


def knn_build_batch(X, offsets, K, S=None, max_iters=12, seed=0, delta=0.001, stop_updates=None,
                    precision=FP32, margin_rel=0.0, ctx=None):
    """NN-Descent lists of several collections in one build (pg_knn_build_batch):
    X holds the collections' rows one after another, collection c being rows
    offsets[c]:offsets[c + 1].  Returns (ids, d2, iters): n x K lists with ids
    local to each collection (each equal to knn_build on the collection's
    rows alone) and each collection's iteration count.  stop_updates (one per
    collection) defaults to delta * n_c * K."""
    import numpy as np
    lib = load_library()
    X = _dev_f32(X, "X")
    n, d = X.shape
    S = (K + 1) // 2 if S is None else S
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    ncoll = len(off) - 1
    if stop_updates is None:
        stop_updates = [int(delta * int(off[c + 1] - off[c]) * K) for c in range(ncoll)]
    stop = np.ascontiguousarray(np.asarray(stop_updates, dtype=np.int64))
    if stop.shape != (ncoll,):
        raise ValueError("stop_updates needs one value per collection")
    p = KnnParams(K=K, S=S, max_iters=max_iters, exact=0, stop_updates=0, seed=seed & (2**64 - 1),
                  precision=precision, margin_rel=float(margin_rel))
    ws_bytes = c_size_t()
    _check(lib.pg_knn_build_batch_workspace(ctypes.byref(p), n, d, ncoll, ctypes.byref(ws_bytes)), "workspace")
    ws = torch.empty(max(ws_bytes.value, 1), dtype=torch.uint8, device=X.device)
    ids = torch.empty((n, K), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, K), dtype=torch.float32, device=X.device)
    iters = np.zeros(ncoll, dtype=np.int32)
    ctx = ctx or context(X.device.index)
    _check(lib.pg_knn_build_batch(ctx.handle, _ptr(X), n, d, X.stride(0), c_void_p(off.ctypes.data), ncoll,
                                  c_void_p(stop.ctypes.data), ctypes.byref(p), _ptr(ws), ws_bytes.value, _ptr(ids),
                                  _ptr(d2), c_void_p(iters.ctypes.data)), "pg_knn_build_batch")
    return ids, d2, iters.tolist()


NOALLOC_WS_BYTES = 128 << 20  # PG_NOALLOC_WS_BYTES of include/pg.h


def knn_build_noalloc(X, K, S=None, max_iters=12, seed=0, stop_updates=None, delta=0.001,
                      bucket_cap=0, chunks=0, precision=FP32, margin_rel=0.0, out=None, ctx=None):
    """knn_build through pg_knn_build_noalloc: the library's static device
    scratch serves as the workspace (no workspace tensor is made).  out
    (optional pair of n x K int32 / float32 device tensors) receives the lists;
    returns (ids, d2, stats dict)."""
    lib = load_library()
    X = _dev_f32(X, "X")
    n, d = X.shape
    S = (K + 1) // 2 if S is None else S
    if stop_updates is None:
        stop_updates = int(delta * n * K)
    p = KnnParams(K=K, S=S, max_iters=max_iters, exact=0, stop_updates=stop_updates,
                  seed=seed & (2**64 - 1), precision=precision, margin_rel=float(margin_rel),
                  bucket_cap=bucket_cap, chunks=chunks)
    if out is None:
        ids = torch.empty((n, K), dtype=torch.int32, device=X.device)
        d2 = torch.empty((n, K), dtype=torch.float32, device=X.device)
    else:
        ids, d2 = out
        if ids.dtype != torch.int32 or d2.dtype != torch.float32 or tuple(ids.shape) != (n, K) \
                or tuple(d2.shape) != (n, K) or not ids.is_contiguous() or not d2.is_contiguous():
            raise ValueError("out must be contiguous n x K int32 and float32 tensors")
    st = KnnStats()
    ctx = ctx or context(X.device.index)
    _check(lib.pg_knn_build_noalloc(ctx.handle, _ptr(X), n, d, X.stride(0), ctypes.byref(p), _ptr(ids),
                                    _ptr(d2), ctypes.byref(st)), "pg_knn_build_noalloc")
    it = st.iters_run
    stats = {"iters": it, "updates": list(st.updates[:it]), "pairs": list(st.pairs[:it]),
             "proposals": list(st.proposals[:it]), "rechecked": list(st.rechecked[:it]),
             "members": list(st.members[:it]), "retries": st.retries, "spilled": st.spilled,
             "join_path": JOIN_PATHS.get(st.join_path, st.join_path)}
    return ids, d2, stats


def exact_knn(X, Q, k, exclude=None, ctx=None):
    """Brute-force k nearest rows of X for every row of Q: returns (ids, d2)."""
    lib = load_library()
    X, Q = _dev_f32(X, "X"), _dev_f32(Q, "Q")
    n, d = X.shape
    nq = Q.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((nq, k), dtype=torch.float32, device=X.device)
    ex = None if exclude is None else _dev_i32(exclude, "exclude")
    ctx = ctx or context(X.device.index)
    _check(lib.pg_exact_knn(ctx.handle, _ptr(X), n, d, X.stride(0), _ptr(Q), nq, Q.stride(0),
                            _ptr(ex), k, _ptr(ids), _ptr(d2)), "pg_exact_knn")
    return ids, d2


def prune(X, cand, R, alpha_deg=60.0, stages=STAGES_ALL, strict_ties=False, pair_d2=None,
          cand_d2=None, precision=FP32, k2p_prev=None, k2p_counts=None, prune_out=False, ctx=None):
    """Refinement of Alg. 2: returns dict(ids, d2, deg, ep, roots).

    cand_d2 (optional, same shape as cand): the canonical squared distances of
    the candidates, e.g. the d2 output of knn_build.  k2p_prev (optional pair
    (ids, deg)): the PRUNE-stage lists of the previous round with the same
    alpha (K2P, Section 5.4; the graph is unchanged); k2p_counts (optional
    int64 device tensor of 2) is added the pairs skipped and tested.  With
    prune_out the dict also holds this call's PRUNE-stage lists
    ("prune_ids", "prune_deg"), the next round's k2p_prev."""
    lib = load_library()
    X = _dev_f32(X, "X")
    cand = _dev_i32(cand, "cand")
    n, d = X.shape
    C = cand.shape[1]
    if cand_d2 is not None:
        cand_d2 = _dev_f32(cand_d2, "cand_d2")
        if tuple(cand_d2.shape) != tuple(cand.shape):
            raise ValueError("cand_d2 must have the shape of cand")
    tab = None
    if pair_d2 is not None:
        tab = pair_d2.contiguous()
        if tab.dtype != torch.float32 or tuple(tab.shape) != (n, C + 1, C + 1):
            raise ValueError("pair_d2 must be float32 of shape (n, C+1, C+1)")
    pi = pd = None
    if prune_out:
        pi = torch.empty((n, R), dtype=torch.int32, device=X.device)
        pd = torch.empty(n, dtype=torch.int32, device=X.device)
    kp_ids = kp_deg = None
    if k2p_prev is not None:
        kp_ids, kp_deg = _dev_i32(k2p_prev[0], "k2p ids"), _dev_i32(k2p_prev[1], "k2p deg")
        if kp_ids.dim() != 2 or kp_ids.shape[0] != n or kp_deg.numel() != n:
            raise ValueError("k2p_prev must be an n x r id tensor and n lengths")
    if k2p_counts is not None and (k2p_counts.dtype != torch.int64 or k2p_counts.numel() < 2
                                   or not k2p_counts.is_cuda):
        raise ValueError("k2p_counts must be a CUDA int64 tensor of 2")
    p = PruneParams(R=R, alpha_deg=float(alpha_deg), stages=stages, strict_ties=int(bool(strict_ties)),
                    pair_d2=tab.data_ptr() if tab is not None else None, precision=precision,
                    k2p_prev_ids=kp_ids.data_ptr() if kp_ids is not None else None,
                    k2p_prev_deg=kp_deg.data_ptr() if kp_deg is not None else None,
                    k2p_prev_R=kp_ids.shape[1] if kp_ids is not None else 0,
                    k2p_counts=k2p_counts.data_ptr() if k2p_counts is not None else None,
                    prune_ids_out=pi.data_ptr() if pi is not None else None,
                    prune_deg_out=pd.data_ptr() if pd is not None else None)
    ws_bytes = c_size_t()
    _check(lib.pg_prune_workspace(ctypes.byref(p), n, d, C, ctypes.byref(ws_bytes)), "workspace")
    ws = torch.empty(max(ws_bytes.value, 1), dtype=torch.uint8, device=X.device)
    g_ids = torch.empty((n, R), dtype=torch.int32, device=X.device)
    g_d2 = torch.empty((n, R), dtype=torch.float32, device=X.device)
    g_deg = torch.empty(n, dtype=torch.int32, device=X.device)
    ep = torch.empty(1, dtype=torch.int32, device=X.device)
    roots = torch.empty(n, dtype=torch.int32, device=X.device)
    nroots = c_int32(0)
    ctx = ctx or context(X.device.index)
    _check(lib.pg_prune(ctx.handle, _ptr(X), n, d, X.stride(0), _ptr(cand),
                        _ptr(cand_d2) if cand_d2 is not None else None, C, ctypes.byref(p),
                        _ptr(ws), ws_bytes.value, _ptr(g_ids), _ptr(g_d2), _ptr(g_deg), _ptr(ep),
                        _ptr(roots), ctypes.byref(nroots)), "pg_prune")
    out = {"ids": g_ids, "d2": g_d2, "deg": g_deg, "ep": ep, "roots": roots[:nroots.value]}
    if prune_out:
        out["prune_ids"], out["prune_deg"] = pi, pd
    return out


def half_rows(X, ctx=None):
    """FP16 copy of the rows of X for search(): returns (X16, exact).  Pass
    X16 to search() only when exact is True."""
    lib = load_library()
    X = _dev_f32(X, "X")
    n, d = X.shape
    ld16 = (d + 7) // 8 * 8
    x16 = torch.empty((n, ld16), dtype=torch.float16, device=X.device)
    flag = torch.empty(1, dtype=torch.int32, device=X.device)
    ctx = ctx or context(X.device.index)
    _check(lib.pg_half_rows(ctx.handle, _ptr(X), n, d, X.stride(0), _ptr(x16), _ptr(flag)), "pg_half_rows")
    return x16, bool(flag.item())


def search(X, g_ids, g_deg, Q, entries, k, L, query_entry=None, exclude=None, record=None,
           pool_out=False, counts=None, x16=None, ctx=None):
    """Alg. 1 beam search for every row of Q: returns (ids, d2), plus the final
    pools (pool_ids, pool_d2), nq x L, when pool_out is set.

    entries: shared entering points; query_entry (nq ids, optional) gives each
    query its own single entering point instead; exclude (nq ids, optional)
    leaves one node out of each query's results.  record (optional pair
    (ids, d2), nq x r): distances of the same query rows recorded by an
    earlier search (its pools), reused instead of gathering rows (P2K,
    Section 5.4); the results do not change.  counts (optional int64 device
    tensor of 2) is added the distances computed and the ones reused.  x16:
    an exact FP16 copy of X from half_rows() (rows gathered at half the
    bytes, results unchanged)."""
    lib = load_library()
    X, Q = _dev_f32(X, "X"), _dev_f32(Q, "Q")
    g_ids, g_deg = _dev_i32(g_ids, "g_ids"), _dev_i32(g_deg, "g_deg")
    n, d = X.shape
    nq = Q.shape[0]
    if entries is not None:
        entries = _dev_i32(entries.reshape(-1), "entries")
    if query_entry is not None:
        query_entry = _dev_i32(query_entry.reshape(-1), "query_entry")
        if query_entry.numel() != nq:
            raise ValueError("query_entry needs one id per query")
    if exclude is not None:
        exclude = _dev_i32(exclude.reshape(-1), "exclude")
        if exclude.numel() != nq:
            raise ValueError("exclude needs one id per query")
    rec_ids = rec_d2 = None
    if record is not None:
        rec_ids, rec_d2 = _dev_i32(record[0], "record ids"), _dev_f32(record[1], "record d2")
        if rec_ids.dim() != 2 or rec_ids.shape[0] != nq or tuple(rec_d2.shape) != tuple(rec_ids.shape):
            raise ValueError("record must be two nq x r tensors")
    if counts is not None and (counts.dtype != torch.int64 or counts.numel() < 2 or not counts.is_cuda):
        raise ValueError("counts must be a CUDA int64 tensor of 2")
    if x16 is not None and (x16.dtype != torch.float16 or tuple(x16.shape) != (n, (d + 7) // 8 * 8)
                            or not x16.is_contiguous() or x16.device != X.device):
        raise ValueError("x16 must be the contiguous (n, d rounded up to 8) float16 copy from half_rows()")
    ids = torch.empty((nq, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((nq, k), dtype=torch.float32, device=X.device)
    pool_ids = pool_d2 = None
    if pool_out:
        pool_ids = torch.empty((nq, L), dtype=torch.int32, device=X.device)
        pool_d2 = torch.empty((nq, L), dtype=torch.float32, device=X.device)
    p = SearchParams(k=k, L=L, n_entry=entries.numel() if entries is not None else 0,
                     entry_ids=entries.data_ptr() if entries is not None else None,
                     query_entry=query_entry.data_ptr() if query_entry is not None else None,
                     exclude=exclude.data_ptr() if exclude is not None else None,
                     record_ids=rec_ids.data_ptr() if rec_ids is not None else None,
                     record_d2=rec_d2.data_ptr() if rec_d2 is not None else None,
                     record_L=rec_ids.shape[1] if rec_ids is not None else 0,
                     pool_ids=pool_ids.data_ptr() if pool_out else None,
                     pool_d2=pool_d2.data_ptr() if pool_out else None,
                     counts=counts.data_ptr() if counts is not None else None,
                     x16=_ptr(x16) if x16 is not None else None)
    ctx = ctx or context(X.device.index)
    _check(lib.pg_search(ctx.handle, _ptr(X), n, d, X.stride(0), _ptr(g_ids), g_ids.shape[1],
                         _ptr(g_deg), _ptr(Q), nq, Q.stride(0), ctypes.byref(p), _ptr(ids), _ptr(d2)),
           "pg_search")
    if pool_out:
        return ids, d2, pool_ids, pool_d2
    return ids, d2


def search_self(X, g_ids, g_deg, k, L, record=None, pool_out=False, counts=None, x16=None, ctx=None):
    """Search phase of OptKCNA (Alg. 5): KANNSearch(G, u, k, L, u) for every
    point u, u not being its own candidate.  Returns (ids, d2), n x k (plus
    the pools with pool_out; record and counts as in search())."""
    n = X.shape[0]
    selfid = torch.arange(n, dtype=torch.int32, device=X.device)
    return search(X, g_ids, g_deg, X, None, k, L, query_entry=selfid, exclude=selfid, record=record,
                  pool_out=pool_out, counts=counts, x16=x16, ctx=ctx)


def opt_kcna(X, cand, k, L, M, alpha_deg, cand_d2=None, record=None, return_pool=False, counts=None,
             x16=None, k2p_prev=None, k2p_counts=None, return_prune=False, ctx=None):
    """OptKCNA (Alg. 5): the alpha-PG of the candidate lists (prune with M and
    alpha, reverse re-prune, connect), then a search from every point on it.
    Returns the new candidate lists (ids, d2), n x k, and with return_pool the
    search pools too (the P2K record of the next round).  k2p_prev: the
    previous round's PRUNE-stage lists (K2P, Section 5.4); with return_prune
    this round's are appended to the result (the next round's k2p_prev)."""
    g = prune(X, cand, M, alpha_deg=alpha_deg, cand_d2=cand_d2, k2p_prev=k2p_prev, k2p_counts=k2p_counts,
              prune_out=return_prune, ctx=ctx)
    r = search_self(X, g["ids"], g["deg"], k, L, record=record, pool_out=return_pool, counts=counts,
                    x16=x16, ctx=ctx)
    r = r if return_pool else (r[0], r[1])
    if return_prune:
        r = tuple(r) + ((g["prune_ids"], g["prune_deg"]),)
    return r


def quality_sample_size(n, eps, l=1):
    """Sample size of the quality examination (Section 5.2): the theorem's
    n_s >= (8 + 2 eps) l log n / eps^2 estimates the mean k-CNA recall within
    eps/2 with probability at least 1 - n^-l."""
    import math
    return int(math.ceil((8.0 + 2.0 * eps) * l * math.log(n) / (eps * eps)))


def quality_examination_async(X, cand, k, sample, ctx=None):
    """Enqueue the quality examination of Section 5.2 on the context's stream
    (pg_quality_examination): returns (estimate, hits) device tensors, the
    estimate being one float64 (the mean over the sampled nodes u of
    |C(u)[:k] & N*_k(u)| / k) and hits the per-node counts.  Read them after
    the context's stream has finished the call."""
    lib = load_library()
    X = _dev_f32(X, "X")
    cand = _dev_i32(cand, "cand")
    n, d = X.shape
    sample = _dev_i32(torch.as_tensor(sample).reshape(-1).to(X.device), "sample")
    ns = sample.numel()
    exact_ids = torch.empty((ns, k), dtype=torch.int32, device=X.device)
    exact_d2 = torch.empty((ns, k), dtype=torch.float32, device=X.device)
    hits = torch.empty(ns, dtype=torch.int32, device=X.device)
    est = torch.empty(1, dtype=torch.float64, device=X.device)
    ctx = ctx or context(X.device.index)
    _check(lib.pg_quality_examination(ctx.handle, _ptr(X), n, d, X.stride(0), _ptr(cand), cand.shape[1], k,
                                      _ptr(sample), ns, _ptr(exact_ids), _ptr(exact_d2), _ptr(hits),
                                      _ptr(est)), "pg_quality_examination")
    return est, hits


def quality_examination(X, cand, k, sample, ctx=None):
    """Estimated k-CNA quality of the candidate lists (Section 5.2), computed
    by pg_quality_examination; waits for the result."""
    ctx = ctx or context(X.device.index)
    est, _ = quality_examination_async(X, cand, k, sample, ctx=ctx)
    ctx.stream.synchronize()
    return float(est.item())


_side_contexts = {}


def _side_context(device):
    """A context on a second stream of the device (default priority), for work
    that overlaps the main stream's (the quality examination)."""
    if device not in _side_contexts:
        _side_contexts[device] = Context(device, torch.cuda.Stream(device=device))
    return _side_contexts[device]


def iter_nsg(X, K, R, k, L, alpha_deg, iterations, S=None, max_iters=12, seed=0, delta=0.001,
             target=None, sample=None, p2k=False, counts=None, half=True, k2p=False, k2p_counts=None,
             ctx=None, **knn_kw):
    """IterNSG (Alg. 6): NN-Descent lists, rounds of OptKCNA with angle
    alpha_deg, then the refinement of Alg. 2 with RNG pruning.  Without
    `target` it runs `iterations` rounds; with `target` the quality
    examination on the nodes `sample` runs before each round and the rounds
    stop once the estimate reaches it (or after `iterations`).  The
    examination runs on a second stream, overlapping the round that follows
    it; that round is dropped when the estimate reaches the target.  Returns the
    graph dict of prune() plus the final candidate lists ("cand", "cand_d2"),
    the rounds run, the estimates and the kNN statistics.  With p2k, every
    round's self-search reuses the distances recorded in the previous round's
    pools (Section 5.4, P2K); the graph is the same.  With k2p, every round's
    prune skips the pairs the previous round's prune settled (Section 5.4,
    K2P; k2p_counts as in prune()); the graph is the same.  counts (optional int64
    device tensor of 2) is added the distances the searches computed and
    reused.  With half (the default), the searches gather rows from an FP16
    copy of X whenever that copy is exact (same results)."""
    cand, cd2, st = knn_build(X, K, S=S, max_iters=max_iters, seed=seed, delta=delta, ctx=ctx, **knn_kw)
    rounds, quality, record = 0, [], None
    x16 = None
    if half and iterations > 0:
        h, exact = half_rows(X, ctx=ctx)
        x16 = h if exact else None
    ctx = ctx or context(X.device.index)
    side, prev_prune = None, None
    while rounds < iterations:
        pending = None
        if target is not None:
            # the examination of the current lists runs on a stream of its own
            # while the next round runs speculatively on the context's stream;
            # the round is dropped when the estimate reaches the target, so the
            # rounds and lists are those of examining first
            if side is None:
                side = _side_context(X.device.index)
            ev = torch.cuda.Event()
            ev.record(ctx.stream)
            side.stream.wait_event(ev)
            with torch.cuda.stream(side.stream):
                est, _ = quality_examination_async(X, cand, k, sample, ctx=side)
            pending = (est, cand)  # cand stays referenced until the estimate is read
        res = opt_kcna(X, cand, k, L, R, alpha_deg, cand_d2=cd2, record=record if p2k else None,
                       return_pool=p2k, counts=counts, x16=x16, k2p_prev=prev_prune if k2p else None,
                       k2p_counts=k2p_counts, return_prune=k2p, ctx=ctx)
        nc, nd = res[0], res[1]
        if p2k:
            pi, pd = res[2], res[3]
        if pending is not None:
            side.stream.synchronize()
            quality.append(float(pending[0].item()))
            if quality[-1] >= target:
                break
        cand, cd2 = nc, nd
        if p2k:
            record = (pi, pd)
        if k2p:
            prev_prune = res[-1]
        rounds += 1
    g = prune(X, cand, R, cand_d2=cd2, ctx=ctx)
    g["cand"], g["cand_d2"], g["knn_stats"] = cand, cd2, st
    g["rounds"], g["quality"] = rounds, quality
    return g


def build_graph(X, K, R, S=None, max_iters=12, seed=0, delta=0.001, alpha_deg=60.0, ctx=None,
                **knn_kw):
    """The whole build path: NN-Descent lists, then prune, reverse, entry point, connect."""
    ids, d2, st = knn_build(X, K, S=S, max_iters=max_iters, seed=seed, delta=delta, ctx=ctx, **knn_kw)
    g = prune(X, ids, R, alpha_deg=alpha_deg, cand_d2=d2, ctx=ctx)
    g["knn_ids"], g["knn_d2"], g["knn_stats"] = ids, d2, st
    return g


# ------------------------------------------------------------------ FastHNSW (Alg. 7)

def hnsw_levels(U, M, ctx=None):
    """Highest layer of every node from its uniform draw U in (0, 1]:
    floor(-ln U / ln M) (Alg. 7, first loop).  Returns (levels int32, m_L)."""
    lib = load_library()
    U = torch.as_tensor(U)
    if U.dtype != torch.float64 or U.dim() != 1 or not U.is_cuda:
        raise ValueError("U must be a 1-D float64 CUDA tensor")
    U = U.contiguous()
    n = U.numel()
    levels = torch.empty(n, dtype=torch.int32, device=U.device)
    top = torch.empty(1, dtype=torch.int32, device=U.device)
    ctx = ctx or context(U.device.index)
    _check(lib.pg_hnsw_levels(ctx.handle, _ptr(U), n, M, _ptr(levels), _ptr(top)), "pg_hnsw_levels")
    return levels, int(top.item())


def _complete_layer(Xi, M, ctx):
    """Every node of a layer with at most M nodes linked to all the others, in
    (d2, id) order (Alg. 7: N(u) = D_i without u)."""
    m = Xi.shape[0]
    ids = torch.full((m, M), -1, dtype=torch.int32, device=Xi.device)
    deg = torch.full((m,), m - 1, dtype=torch.int32, device=Xi.device)
    if m >= 2:
        self_ids = torch.arange(m, dtype=torch.int32, device=Xi.device)
        nb, _ = exact_knn(Xi, Xi, m - 1, exclude=self_ids, ctx=ctx)
        ids[:, :m - 1] = nb
    return ids, deg


def opt_hnsw(X, U, k0, ef, M, alpha_deg, iterations=2, S=None, max_iters=12, seed=0, delta=0.001,
             p2k=False, ctx=None, **knn_kw):
    """OptHNSW (Alg. 7): layers from the draws U, then every layer D_i with
    more than M nodes built by IterNSG(D_i, k0, ef, ef, M, alpha) on its own
    rows, smaller layers as complete graphs; the entry point is the smallest
    id of the top layer.  In each layer's OptKCNA search the pool holds
    L = ef entries and C(u) takes the ef - 1 of them other than u; NN-Descent
    uses K = min(k0, |D_i| - 1) and stops after delta |D_i| K updates.
    Returns dict(levels, max_level, ep, layers); layer i holds its nodes
    (global ids, ascending), pos (global -> local id, -1 outside), X (its
    rows), ids / deg (the graph in local ids)."""
    X = _dev_f32(X, "X")
    n = X.shape[0]
    ctx = ctx or context(X.device.index)
    levels, top = hnsw_levels(U, M, ctx=ctx)
    layers = []
    for i in range(top + 1):
        nodes = torch.nonzero(levels >= i).flatten().to(torch.int32) if i else \
            torch.arange(n, dtype=torch.int32, device=X.device)
        m = nodes.numel()
        Xi = X if i == 0 else X[nodes.long()].contiguous()
        if m <= M:
            ids, deg = _complete_layer(Xi, M, ctx)
        else:
            K = min(k0, m - 1)
            Si = min((K + 1) // 2 if S is None else S, K)
            g = iter_nsg(Xi, K, M, ef - 1, ef, alpha_deg, iterations, S=Si, max_iters=max_iters,
                         seed=seed, stop_updates=int(delta * m * K), p2k=p2k, ctx=ctx, **knn_kw)
            ids, deg = g["ids"], g["deg"]
        pos = torch.full((n,), -1, dtype=torch.int32, device=X.device)
        pos[nodes.long()] = torch.arange(m, dtype=torch.int32, device=X.device)
        layers.append({"nodes": nodes, "pos": pos, "X": Xi, "ids": ids, "deg": deg})
    ep = int(layers[top]["nodes"][0].item())
    return {"levels": levels, "max_level": top, "ep": ep, "layers": layers}


def hnsw_search(H, Q, k, ef, ctx=None):
    """k-ANN search on a layered graph: greedy routing (KANNSearch with
    k = L = 1) from the entry point down to layer 1, each layer entered at
    the node found above it, then KANNSearch with L = ef on layer 0.
    Returns (ids, d2), nq x k, ids global."""
    layers = H["layers"]
    Q = _dev_f32(Q, "Q")
    nq = Q.shape[0]
    w = torch.full((nq,), H["ep"], dtype=torch.int32, device=Q.device)
    for i in range(H["max_level"], 0, -1):
        L_ = layers[i]
        e = L_["pos"][w.long()].contiguous()
        f, _ = search(L_["X"], L_["ids"], L_["deg"], Q, None, 1, 1, query_entry=e, ctx=ctx)
        w = L_["nodes"][f[:, 0].long()].contiguous()
    L0 = layers[0]
    return search(L0["X"], L0["ids"], L0["deg"], Q, None, k, ef, query_entry=w, ctx=ctx)
