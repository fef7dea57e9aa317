"""Benchmark of the proximity-graph build path on one MI355X.

One step = one pass of the whole hot path over the resident input: the
NN-Descent kNN lists, prune, reverse re-prune, entry point and connect (the
graph build), then beam search of the query batch.  Inputs are in HBM before
the timed region starts.

The default run is the suite: the GIST-shaped 1M x 960 set is the headline
(plain FP32 against FP16-MFMA tiles with FP32 recheck, timed over --steps),
then the Deep-shaped 10M x 96 set (FP32 against BF16), the SIFT-shaped
1M x 128 set (FP32 against FP16) and the tiny 10k x 128 set as legs timed
over min(--steps, --leg-steps).  --workload NAME runs one set alone.

Search entering points: Alg. 1 enters at the single point ep.  The recall
ladder is reported for {ep} alone, for ep plus a seeded uniform sample of E
ids (E = 256, 1024, 4096; the same ids for every path), and for ep plus
every connect root.  Each ladder stops at the smallest L whose recall@10
reaches 0.95 (measured once, before timing, against GPU brute force); the
timed search takes, among the sets that reached it, the one that evaluates
the fewest distances per query (entries + L R at most).

Prints ONE JSON line.  `value` is the headline set's build throughput in
points/s over the timed steps (search included in the step) on its fastest
path that reaches the recall target.  `roofline` reports the join kernel (the
dominant one) from HIP events on the library's stream.  `cpu_baseline` times
the FP64 oracle on a bounded sample of the headline set on the host cores,
with a one-core run of the whole tiny set beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SUITE = ["gist1m", "deep10m", "sift1m", "tiny"]  # headline first
ENTRY_SAMPLES = [256, 1024, 4096]
WORKLOADS = {
    # SIFT-shaped: 1M x 128, 100 Gaussian clusters (sigma 20) rounded to [0,255]
    "sift1m": dict(n=1_000_000, nq=10_000, d=128, K=64, R=32, S=32, iters=12, seed=2, paths="fp32,fp16",
                   cpu_sample=100_000,
                   gen="sift_like", desc="sift-like 1Mx128 mixture-of-100, K=64 R=32 FP32"),
    # GIST-shaped precision mode: 1M x 960 float data (Gamma(2, 0.05) + 50 offsets);
    # the FP16 path is the mixed one (16-bit tiles prefilter, FP32 recheck)
    "gist1m": dict(n=1_000_000, nq=1_000, d=960, K=64, R=32, S=32, iters=12, seed=3, paths="fp32,fp16",
                   cpu_sample=30_000,
                   gen="gist_like", desc="gist-like 1Mx960 Gamma(2,0.05)+50 offsets, K=64 R=32 FP32 storage"),
    # Deep-shaped: 10M x 96 unit vectors, 1000 Gaussian clusters; BF16 tiles with
    # FP32 recheck against plain FP32
    "deep10m": dict(n=10_000_000, nq=10_000, d=96, K=64, R=32, S=32, iters=12, seed=4, paths="fp32,bf16",
                    cpu_sample=50_000,
                    gen="unit_mixture", desc="deep-like 10Mx96 unit mixture-of-1000, K=64 R=32 FP32 storage"),
    # tiny: 10k x 128 integers
    "tiny": dict(n=10_000, nq=100, d=128, K=32, R=32, S=16, iters=12, seed=0, paths="fp32",
                 cpu_sample=10_000,
                 gen="uniform_int", desc="uniform-int 10kx128, K=32 R=32 FP32"),
}
SERVE_BATCH = 16  # builds of one shape the serving loop runs as one batched build
# knobs of the build (bucket capacity, first-iteration passes) the autotuner
# chose for each set and join precision on one MI355X (`--tune` writes it);
# they change the speed of a build, never its lists
TUNE_CACHE = os.path.join(ROOT, "paper_2410_01231_amd", "tune_cache.json")
L_LADDER = [16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048]
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector and FP32 MFMA (dense)
PEAK_16BIT_TFLOPS = 2500.0  # MI355X dense FP16 / BF16 MFMA
PEAK_HBM_GBS = 8000.0
# HBM traffic of the join measured with rocprofv3 counters; only valid while
# the join source is the one the counters were taken on (sha256 recorded)
JOIN_SOURCE = os.path.join(ROOT, "paper_2410_01231_amd", "csrc", "knn.hip")


def measured_traffic(path_name, workload):
    """HBM bytes per join launch for this path from the counter summary of the
    workload (profiles/traffic_join_<workload>.md), or None."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", f"traffic_join_{workload}.md")).read()
        sha = hashlib.sha256(open(JOIN_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"join source sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != sha:
        return None
    m = re.search(r"^traffic_bytes_per_launch\[" + re.escape(path_name) + r"\]: ([0-9.e+]+)$", text, re.M)
    return float(m.group(1)) if m else None


# issue ceiling of the FP32 direct form without packed FP32: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz lane instructions/s, two instructions (subtract, FMA) per
# pair and dimension counted as 3 flops
DIRECT_FORM_CEILING_TFLOPS = 256 * 4 * 16 * 2.4e9 * 1.5 / 1e12


def compulsory_bytes(st, n, d, K, S, sixteen):
    """Bytes an NN-Descent build must move at least: per iteration the rows
    once (FP32, or the 16-bit copy), the lists read and written, the sampled
    and reverse sets written and read, and 12 bytes per proposal."""
    row = 2 * ((d + 15) // 16 * 16) if sixteen else 4 * d
    fixed = n * row + 2 * n * K * 8 + 2 * n * (2 * S + K + S) * 4
    return sum(fixed + 12 * p for p in st["proposals"][:st["iters"]])


def roofline(join_path, work, launches, total_ms, name, workload):
    """Roofline entry of the join kernel: flops or bytes per launch over its mean duration."""
    avg_ms = total_ms / max(launches, 1)
    per_launch = work / max(launches, 1)
    if join_path.endswith("mfma") and join_path.startswith("fp32"):
        bound, unit, peak, scale = "mfma", "TFLOP/s", PEAK_FP32_TFLOPS, 1e12
    elif join_path == "fp32-valu":
        bound, unit, peak, scale = "alu", "TFLOP/s", PEAK_FP32_TFLOPS, 1e12
    else:
        bound, unit, peak, scale = "hbm", "GB/s", PEAK_HBM_GBS, 1e9
    achieved = per_launch / (avg_ms / 1000.0) / scale if launches else 0.0
    out = {"kernel": "join", "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
           "frac": achieved / peak,
           "traffic": measured_traffic(name, workload),
           "work_per_launch": per_launch,
           "work_unit": "flops" if scale == 1e12 else "bytes",
           "avg_launch_ms": avg_ms, "launches": launches}
    if join_path == "fp32-valu":
        out["issue_ceiling"] = DIRECT_FORM_CEILING_TFLOPS
        out["frac_of_issue_ceiling"] = achieved / DIRECT_FORM_CEILING_TFLOPS
    return out


def mfma_utilisation(join_path, pairs, d, join_ms):
    """Dense MFMA rate of the join's Gram tiles (2 d16 flops per pair for the
    16-bit tiles, 2 d for the FP32 ones) against the chip's peak for that type."""
    if not join_path.endswith(("mfma", "mixed")) or join_ms <= 0:
        return None
    d16 = (d + 15) // 16 * 16
    sixteen = not join_path.startswith("fp32")
    flops = 2.0 * pairs * (d16 if sixteen else d)
    peak = PEAK_16BIT_TFLOPS if sixteen else PEAK_FP32_TFLOPS
    rate = flops / (join_ms / 1000.0) / 1e12
    return {"tflops": rate, "peak_tflops": peak, "frac": rate / peak,
            "dtype": "f32" if not sixteen else join_path.split("-")[0]}


def gen_data(w):
    from paper_2410_01231_amd import datagen
    if w["gen"] == "sift_like":
        return datagen.sift_like(w["n"], w["nq"], d=w["d"], seed=w["seed"])
    if w["gen"] == "gist_like":
        return datagen.gist_like(w["n"], w["nq"], d=w["d"], seed=w["seed"])
    if w["gen"] == "unit_mixture":
        return datagen.unit_mixture(w["n"], w["nq"], d=w["d"], seed=w["seed"])
    X = datagen.uniform_int(w["n"], w["d"], seed=w["seed"])
    Q = datagen.uniform_int(w["nq"], w["d"], seed=w["seed"] + 1)
    return X, Q


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recall(found, gt):
    k = gt.shape[1]
    f = found[:, :k]
    hits = 0
    for a, b in zip(f, gt):
        hits += len(set(a[a >= 0].tolist()) & set(b.tolist()))
    return hits / gt.size


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_build_time(w, X, budget_n):
    """The oracle (as it stands): NN-Descent + refine of the first budget_n points."""
    from oracle import oracle as O
    Xs = np.ascontiguousarray(X[:budget_n])
    stop = int(0.001 * budget_n * w["K"])
    t0 = time.perf_counter()
    ids, _, _, st = O.nndescent(Xs, w["K"], w["S"], w["iters"], 1, stop_updates=stop)
    O.refine(Xs, ids, w["R"])
    return time.perf_counter() - t0, st["iters"]


def cpu_baseline(name, w, X, budget_n):
    """The oracle on a bounded sample of the workload on every host core, and
    on one core over the whole tiny set (a child process with one OpenMP thread)."""
    dt, iters = oracle_build_time(w, X, budget_n)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": budget_n / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"first {budget_n} points of the {name} set: NN-Descent ({iters} iters) + "
                     f"refine (prune, reverse, entry point, connect), {dt:.1f} s"}
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-core"], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode == 0 and r.stdout.strip():
        out["one_core_tiny"] = json.loads(r.stdout.strip().splitlines()[-1])
    else:
        out["one_core_tiny"] = {"error": r.stderr[-400:]}
    return out


def oracle_one_core():
    """Child process of cpu_baseline: the whole tiny set through the oracle."""
    w = WORKLOADS["tiny"]
    X, _ = gen_data(w)
    dt, iters = oracle_build_time(w, X, w["n"])
    print(json.dumps({"value": w["n"] / dt, "unit": "points/s", "cores": 1, "seconds": dt,
                      "sample": f"the whole tiny set ({w['n']} points): NN-Descent ({iters} iters) + refine"}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="suite", choices=["suite"] + sorted(WORKLOADS))
    ap.add_argument("--leg-steps", type=int, default=2,
                    help="timed steps of the suite's legs (at most --steps)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="points of the oracle's bounded sample (0: the workload's default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-one-core", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--iternsg", type=int, default=0, metavar="I",
                    help="also build the IterNSG graph (Alg. 6) with I OptKCNA rounds on the "
                         "fastest path and report its build time and search recall")
    ap.add_argument("--hnsw", type=int, default=0, metavar="EF",
                    help="also build the global HNSW (Alg. 7, FastHNSW) with ef=EF, M=R, k0=K, "
                         "alpha 65 degrees and 2 OptKCNA rounds per layer on the fastest path, "
                         "and report its build time and layered-search recall")
    ap.add_argument("--serve", type=int, default=0, metavar="JOBS",
                    help="also run the serving mix: JOBS collections (N log-uniform in [1e3, 2e5], "
                         "d in {96, 128, 384, 768}, unit vectors in 20 clusters, K = R = 32) with 4 "
                         "query batches each, first saturated, then Poisson arrivals at 0.5 and 0.9 times that rate")
    ap.add_argument("--serve-budget-gb", type=float, default=48.0)
    ap.add_argument("--paths", default="",
                    help="comma-separated join paths of a single --workload run: fp32, fp16, bf16, "
                         "fp32-valu, fp16-stated (default: the workload's own)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the "
                         "HBM byte counters against a copy of known size) and exit")
    ap.add_argument("--tune", action="store_true",
                    help="only tune the build knobs of the suite's sets (or --workload) per join "
                         "precision into --tune-cache and exit")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, metavar="PATH")
    ap.add_argument("--default-knobs", action="store_true",
                    help="build with the library's default knobs, not the tuned ones")
    args = ap.parse_args()
    global TUNED
    TUNED = not args.default_knobs
    if args.oracle_one_core:
        oracle_one_core()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5,
                          "expected_read_bytes_per_copy": nbytes,
                          "expected_write_bytes_per_copy": nbytes}), flush=True)
        return
    from paper_2410_01231_amd import pg
    torch.cuda.set_device(0)
    ctx = pg.context(0)
    if args.tune:
        run_tune(args, pg, torch, ctx)
        return

    names = SUITE if args.workload == "suite" else [args.workload]
    legs = {}
    head_name = names[0]
    head_X = None
    for i, name in enumerate(names):
        steps = args.steps if i == 0 else max(1, min(args.steps, args.leg_steps))
        warmup = args.warmup if i == 0 else 1
        paths = args.paths if (args.paths and args.workload != "suite") else WORKLOADS[name]["paths"]
        res, X = run_workload(args, name, paths, steps, warmup, pg, torch, ctx, keep_x=(i == 0))
        legs[name] = res
        if i == 0:
            head_X = X
        torch.cuda.empty_cache()
    head = legs[head_name]
    r = head["paths"][head["best"]]
    w = WORKLOADS[head_name]
    out = {
        "metric": "build points/s at search recall@10>=0.95, FP32 vs FP16-MFMA; query p50/p99",
        "value": r["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1, "steps": head["steps"], "warmup": head["warmup"],
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": PATHS[head["best"]]["dtype"], "data": "synthetic",
        "config": {"workload": w["desc"], "n": w["n"], "d": w["d"], "K": w["K"], "R": w["R"], "S": w["S"],
                   "max_iters": w["iters"], "delta": 0.001, "nq": w["nq"], "k": 10,
                   "L": r["L"], "entries": r["entries"], "path": head["best"]},
        "recall@10": r["recall@10"], "recall@10_ep_only": r["recall_ep_only"],
        "knn_recall_sample": r["knn_recall_sample"],
        "qps_batch": r["qps_batch"], "query_latency_ms_batch1": r["query_latency_ms_batch1"],
        "roofline": r["roofline"],
        "mfma_utilisation": r["mfma_utilisation"],
        "fp32_vs_mixed": {p: {"points_per_s": v["points_per_s"], "ms_per_step": v["ms_per_step"],
                              "recall@10": v["recall@10"], "join_path": v["join_path"]}
                          for p, v in head["paths"].items()},
        "host_upload": head["host_upload"],
        "workloads": legs,
    }
    if args.iternsg or args.hnsw or args.serve:
        Xd = torch.from_numpy(head_X).cuda()
        X, Q = gen_data(w)
        Qd = torch.from_numpy(Q).cuda()
        gt, _ = pg.exact_knn(Xd, Qd, 10, ctx=ctx)
        gt = gt.cpu().numpy()
        if args.iternsg:
            out["iter_nsg"] = run_iternsg(args, w, pg, torch, ctx, Xd, Qd, gt, PATHS[head["best"]])
        if args.hnsw:
            out["fast_hnsw"] = run_hnsw(args, w, pg, torch, ctx, Xd, Qd, gt, PATHS[head["best"]])
        if args.serve:
            out["serving"] = run_serve(args)
    if not args.no_cpu_baseline:
        budget = args.cpu_sample or w["cpu_sample"]
        log(f"[bench] cpu baseline on {budget} points of {head_name}")
        out["cpu_baseline"] = cpu_baseline(head_name, w, head_X, budget)
    print(json.dumps(out), flush=True)


def run_workload(args, name, paths, steps, warmup, pg, torch, ctx, keep_x=False):
    """One workload: every path timed over `steps` steps after `warmup` builds."""
    w = WORKLOADS[name]
    log(f"[bench] generating {w['desc']}")
    X, Q = gen_data(w)
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    n, K = w["n"], w["K"]
    gt, _ = pg.exact_knn(Xd, Qd, 10, ctx=ctx)
    gt = gt.cpu().numpy()
    samp = np.random.default_rng(9).choice(n, size=min(n, 2000), replace=False).astype(np.int32)
    samp_d = torch.from_numpy(samp).cuda()
    kt, _ = pg.exact_knn(Xd, Xd[samp_d.long()], K, exclude=samp_d, ctx=ctx)
    kt = kt.cpu().numpy()

    # the upload of X over PCIe, reported beside the HBM-resident build rate
    # (the library takes device pointers, so it is never part of `value`)
    Xh = torch.from_numpy(X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tmp = Xh.cuda()
    torch.cuda.synchronize()
    up_pageable = time.perf_counter() - t0
    Xp = Xh.pin_memory()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tmp = Xp.to("cuda", non_blocking=True)
    torch.cuda.synchronize()
    up_pinned = time.perf_counter() - t0
    del tmp, Xp
    log(f"[bench] upload of X ({X.nbytes / 1e9:.2f} GB): pageable {1000 * up_pageable:.1f} ms, "
        f"pinned {1000 * up_pinned:.1f} ms")

    results = {}
    for path in paths.split(","):
        results[path] = run_path(steps, warmup, w, pg, torch, ctx, Xd, Qd, gt, kt, samp, PATHS[path], name)
    # kNN-list entries and graph edges that differ from the FP32 build
    ref = next((results[p] for p in ("fp32", "fp32-valu") if p in results), None)
    for p in results:
        if ref is not None and results[p] is not ref:
            results[p]["knn_entries_differing_from_fp32"] = int((results[p]["_ids"] != ref["_ids"]).sum())
            results[p]["graph_edges_differing_from_fp32"] = int((results[p]["_graph"] != ref["_graph"]).sum())
    for p in results:
        results[p].pop("_ids")
        results[p].pop("_graph")
    ok = [p for p in results if results[p]["recall@10"] >= 0.95] or list(results)
    best = max(ok, key=lambda p: results[p]["points_per_s"])
    up = {"bytes": int(X.nbytes), "pageable_ms": 1000.0 * up_pageable, "pinned_ms": 1000.0 * up_pinned,
          "points_per_s_with_pinned_upload": n / (results[best]["ms_per_step"] / 1000.0 + up_pinned)}
    del Xd, Qd
    return ({"workload": w["desc"], "steps": steps, "warmup": warmup, "best": best, "paths": results,
             "host_upload": up}, X if keep_x else None)


def run_iternsg(args, w, pg, torch, ctx, Xd, Qd, gt, path):
    """IterNSG (Alg. 6) with args.iternsg OptKCNA rounds (alpha 65 degrees, k = K,
    L = 2K): build time without P2K and K2P (the reported one), with P2K and
    with K2P (Section 5.4; the graphs must be identical), each after an
    untimed warm-up, then the search ladders."""
    K, R, S = w["K"], w["R"], w["S"]

    def build(opt, counts=None):
        return pg.iter_nsg(Xd, K, R, K, 2 * K, 65.0, args.iternsg, S=S, max_iters=w["iters"], seed=1,
                           delta=0.001, precision=path["precision"], p2k=opt == "p2k",
                           counts=counts if opt != "k2p" else None,
                           k2p=opt == "k2p", k2p_counts=counts if opt == "k2p" else None, ctx=ctx)
    times, graphs, counts = {}, {}, {}
    for opt in ("none", "p2k", "k2p"):
        build(opt)
        torch.cuda.synchronize()
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        t0 = time.perf_counter()
        graphs[opt] = build(opt, cnt)
        torch.cuda.synchronize()
        times[opt] = time.perf_counter() - t0
        counts[opt] = [int(x) for x in cnt.cpu().tolist()]
        log(f"[bench] iternsg {opt} build {times[opt]:.3f} s, counts {counts[opt]}")
    same = {o: all(torch.equal(graphs["none"][k], graphs[o][k]) for k in ("ids", "deg", "cand"))
            for o in ("p2k", "k2p")}
    g = graphs["none"]
    build_s = times["none"]
    ladders, sizes, sets = {}, {}, {}
    for sname, ent in entry_sets(g, w["n"], torch):
        lad = ladder(pg, torch, ctx, Xd, g, Qd, gt, ent, None)
        ladders[sname], sizes[sname], sets[sname] = lad, int(ent.numel()), ent
        log(f"[bench] iternsg entries {sname}: {lad}")
    ename, chosen, _ = pick_entries(ladders, sizes, R)
    entries = sets[ename]
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    pg.search(Xd, g["ids"], g["deg"], Qd, entries, 10, chosen or L_LADDER[-1], ctx=ctx)
    s1.record()
    s1.synchronize()
    return {"rounds": args.iternsg, "alpha_deg": 65.0, "k": K, "L_search": 2 * K,
            "build_ms": 1000.0 * build_s, "points_per_s": w["n"] / build_s,
            "build_ms_with_p2k": 1000.0 * times["p2k"], "build_ms_with_k2p": 1000.0 * times["k2p"],
            "self_search_distances": {"without_p2k": counts["none"][0],
                                      "with_p2k_computed": counts["p2k"][0],
                                      "with_p2k_reused": counts["p2k"][1]},
            "k2p_pairs": {"skipped": counts["k2p"][0], "tested": counts["k2p"][1]},
            "p2k_graph_identical": bool(same["p2k"]), "k2p_graph_identical": bool(same["k2p"]),
            "L": chosen, "entries": ename, "search_ladders": ladders,
            "qps_batch": Qd.shape[0] / (s0.elapsed_time(s1) / 1000.0)}


def run_hnsw(args, w, pg, torch, ctx, Xd, Qd, gt, path):
    """FastHNSW (Alg. 7): layers drawn from seeded uniforms, each layer built by
    IterNSG with ef = args.hnsw, M = R, k0 = K, alpha 65 degrees, 2 rounds;
    build time (untimed warm-up first), then the layered-search ladder."""
    from paper_2410_01231_amd import datagen
    K, R, S, ef = w["K"], w["R"], w["S"], args.hnsw
    U = torch.from_numpy(datagen.uniform_open01(w["n"], seed=7)).cuda()

    def build():
        return pg.opt_hnsw(Xd, U, K, ef, R, 65.0, iterations=2, S=S, max_iters=w["iters"], seed=1,
                           delta=0.001, precision=path["precision"], ctx=ctx)
    build()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = build()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    ladder, chosen = [], None
    for L in L_LADDER:
        f, _ = pg.hnsw_search(H, Qd, 10, L, ctx=ctx)
        r = recall(f.cpu().numpy(), gt)
        ladder.append((L, r))
        log(f"[bench] hnsw ef_search={L} recall@10={r:.4f}")
        if r >= 0.95:
            chosen = L
            break
    Ls = chosen or L_LADDER[-1]
    pg.hnsw_search(H, Qd, 10, Ls, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pg.hnsw_search(H, Qd, 10, Ls, ctx=ctx)
    torch.cuda.synchronize()
    qs = time.perf_counter() - t0
    sizes = [int(l["nodes"].numel()) for l in H["layers"]]
    return {"ef": ef, "M": R, "k0": K, "alpha_deg": 65.0, "rounds": 2, "layer_sizes": sizes,
            "build_ms": 1000.0 * build_s, "points_per_s": w["n"] / build_s, "ef_search": chosen,
            "search_ladder": ladder, "qps_batch": Qd.shape[0] / qs}


def run_serve(args):
    """The serving mix (continuous batching of build jobs and query batches,
    admission by HBM footprint): saturated throughput, then latencies under
    Poisson arrivals at 0.5 and 0.9 times the saturated job rate."""
    from paper_2410_01231_amd import datagen
    from paper_2410_01231_amd.serve import BuildJob, QueryBatch, Server, percentiles
    rng = np.random.default_rng(5)
    jobs, batches = [], []
    for i in range(args.serve):
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
        d = int(rng.choice([96, 128, 384, 768]))
        sizes = rng.integers(1, 513, size=4)
        X, Q = datagen.unit_mixture(n, int(sizes.sum()), d=d, n_clusters=20, seed=100 + i)
        jobs.append(BuildJob(f"j{i}", X, K=32, R=32, S=16, max_iters=12, seed=1))
        cuts = np.concatenate([[0], np.cumsum(sizes)])
        batches.append([QueryBatch(f"j{i}", Q[cuts[b]:cuts[b + 1]], k=10, L=64) for b in range(4)])
    points = sum(j.X.shape[0] for j in jobs)
    log(f"[bench] serving mix: {len(jobs)} jobs, {points} points")
    budget = int(args.serve_budget_gb * (1 << 30))

    def run(arrivals, batch):
        srv = Server(budget, workers=8, batch_builds=batch)
        done_q = {j.job_id: 0 for j in jobs}
        lock = threading.Lock()

        def query_done(job_id):
            def cb(_):
                with lock:
                    done_q[job_id] += 1
                    last = done_q[job_id] == 4
                if last:
                    srv.release(job_id)
            return cb
        fb, fq = [], []
        t0 = time.perf_counter()
        for j, qs, at in zip(jobs, batches, arrivals):
            delay = t0 + at - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            fb.append(srv.submit_build(j))
            for q in qs:
                f = srv.submit_query(q)
                f.add_done_callback(query_done(j.job_id))
                fq.append(f)
        blat = [f.result()[1].latency for f in fb]
        qres = [f.result()[1] for f in fq]
        wall = time.perf_counter() - t0
        srv.close()
        log(f"[bench] serving run (batch {batch}): {wall:.2f} s, peak ledger {srv.peak_in_use / 2**30:.1f} GiB, "
            f"{len(srv.batch_log)} batched builds")
        return wall, blat, qres, srv.peak_in_use

    def ms(v):
        return {k: (1000.0 * x if x is not None else None) for k, x in percentiles(v).items()}

    # saturated: everything submitted at once, builds one by one and batched
    wall1, _, _, peak = run([0.0] * len(jobs), 1)
    wall, _, _, peakb = run([0.0] * len(jobs), SERVE_BATCH)
    peak = max(peak, peakb)
    rate = len(jobs) / wall
    loads = []
    for load in (0.5, 0.9):
        gaps = rng.exponential(1.0 / (load * rate), size=len(jobs))
        wall2, blat, qres, peak2 = run(np.cumsum(gaps) - gaps[0], SERVE_BATCH)
        peak = max(peak, peak2)
        loads.append({"load": load, "arrival_rate_jobs_per_s": load * rate, "wall_s": wall2,
                      "build_latency_ms": ms(blat), "query_latency_ms": ms([t.latency for t in qres]),
                      "query_service_ms": ms([t.service for t in qres])})
        log(f"[bench] serving at {load} x saturated rate: build p50/p99 {loads[-1]['build_latency_ms']}")
    return {"jobs": len(jobs), "points": points, "budget_bytes": budget, "batch_builds": SERVE_BATCH,
            "saturated_s_one_by_one": wall1, "saturated_points_per_s_one_by_one": points / wall1,
            "saturated_s": wall, "saturated_jobs_per_s": rate, "saturated_points_per_s": points / wall,
            "peak_in_use_bytes": peak, "poisson": loads}


# join paths: precision code of pg_knn_build, dtype the join computes in
PATHS = {
    "fp32": {"name": "fp32", "precision": 0, "dtype": "f32"},
    "fp16": {"name": "fp16", "precision": 1, "dtype": "f16-mfma/f32-acc"},
    "bf16": {"name": "bf16", "precision": 2, "dtype": "bf16-mfma/f32-acc"},
    "fp32-valu": {"name": "fp32-valu", "precision": 3, "dtype": "f32"},
    # the precision mode as stated: FP16 tiles, FP32 recheck within a 1e-3
    # relative margin of the cut only (not rigorous on float data)
    "fp16-stated": {"name": "fp16-stated", "precision": 1, "dtype": "f16-mfma/f32-acc", "margin_rel": -1e-3},
}


def ladder(pg, torch, ctx, Xd, g, Qd, gt, entries, x16, stop=0.95):
    """Recall@10 over L_LADDER until it reaches `stop`: [(L, recall)]."""
    out = []
    for L in L_LADDER:
        f, _ = pg.search(Xd, g["ids"], g["deg"], Qd, entries, 10, L, x16=x16, ctx=ctx)
        r = recall(f.cpu().numpy(), gt)
        out.append((L, r))
        if r >= stop:
            break
    return out


def entry_sets(g, n, torch):
    """The entering-point sets in the order the search tries them: {ep}, ep
    plus seeded uniform samples of E ids, ep plus every connect root."""
    from paper_2410_01231_amd import datagen
    sets = [("ep", g["ep"])]
    for E in ENTRY_SAMPLES:
        if E < n:
            ids = torch.from_numpy(datagen.entry_sample(n, E)).to(g["ep"].device)
            sets.append((f"ep+{E} seeded", torch.cat([g["ep"], ids]).contiguous()))
    sets.append(("ep+roots", torch.cat([g["ep"], g["roots"]]).contiguous()))
    return sets


def pick_entries(ladders, sizes, R):
    """Among the entering-point sets whose ladder reached recall@10 >= 0.95,
    the one whose search evaluates the fewest distances per query (entries
    plus L R neighbours at most); if none reached it, the last set at its
    widest beam.  Returns (set name, L, recall)."""
    ok = [(sizes[s] + lad[-1][0] * R, s) for s, lad in ladders.items() if lad[-1][1] >= 0.95]
    s = min(ok)[1] if ok else list(ladders)[-1]
    return s, ladders[s][-1][0], ladders[s][-1][1]


def run_path(steps, warmup, w, pg, torch, ctx, Xd, Qd, gt, kt, samp, path, name):
    n, K, R, S = w["n"], w["K"], w["R"], w["S"]
    prec = path["precision"]
    last = {}

    knobs = tuned_knobs(pg, ctx, Xd, w, prec) if TUNED else None
    log(f"[bench] {name} {path['name']} knobs {knobs or 'default'}")
    kn = {k: v for k, v in (knobs or {}).items() if k != "precision"}

    def build():
        ids, d2, st = pg.knn_build(Xd, K, S=S, max_iters=w["iters"], seed=1, delta=0.001,
                                   precision=prec, margin_rel=path.get("margin_rel", 0.0), ctx=ctx, **kn)
        g = pg.prune(Xd, ids, R, cand_d2=d2, ctx=ctx)
        last["d2"] = d2
        return ids, st, g

    # ---- warm-up and recall calibration (untimed)
    for i in range(max(warmup, 1)):
        t0 = time.perf_counter()
        ids, st, g = build()
        torch.cuda.synchronize()
        log(f"[bench] {name} {path['name']} warmup {i}: {time.perf_counter() - t0:.3f} s, iters {st['iters']}, "
            f"join {st['join_path']}, roots {len(g['roots'])}, retries {st['retries']}, "
            f"spilled {st['spilled']}")
        log(f"[bench]   updates {st['updates']}\n[bench]   pairs {st['pairs']}\n"
            f"[bench]   proposals {st['proposals']}\n[bench]   rechecked {st['rechecked']}")
    # rows for the search: an FP16 copy when it holds X exactly (same results)
    h16, exact16 = pg.half_rows(Xd, ctx=ctx)
    x16 = h16 if exact16 else None
    ladders, sizes = {}, {}
    for sname, ent in entry_sets(g, n, torch):
        lad = ladder(pg, torch, ctx, Xd, g, Qd, gt, ent, x16)
        ladders[sname], sizes[sname] = lad, int(ent.numel())
        log(f"[bench] {name} {path['name']} entries {sname} ({ent.numel()}): {lad}")
    ename, L_ch, rec = pick_entries(ladders, sizes, R)
    n_entry_seeded = int(ename.split("+")[1].split()[0]) if "seeded" in ename else 0

    def entries_of(g):
        from paper_2410_01231_amd import datagen
        if ename == "ep":
            return g["ep"]
        if n_entry_seeded:
            return torch.cat([g["ep"], torch.from_numpy(datagen.entry_sample(n, n_entry_seeded)).cuda()])
        return torch.cat([g["ep"], g["roots"]]).contiguous()
    entries = entries_of(g)
    kl = ids.cpu().numpy()[samp]
    knn_recall = float(np.mean([len(set(a) & set(b)) / K for a, b in zip(kl, kt)]))
    # distance error of the stored list distances against FP64 (first 200 sampled nodes)
    sub = torch.from_numpy(samp[:200]).cuda().long()
    xs = Xd[sub].double()
    kl_d2 = last["d2"].double()[sub]
    nb = Xd[ids[sub].long()].double()
    exact = ((xs[:, None, :] - nb) ** 2).sum(-1)
    rel = ((kl_d2 - exact).abs() / exact.clamp_min(1e-300)).flatten()
    d2_err = {"max": float(rel.max()), "median": float(rel.median())}

    # ---- timed steps
    ctx.set_timing(True)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ids, st, g = build()
        h16, exact16 = pg.half_rows(Xd, ctx=ctx)
        pg.search(Xd, g["ids"], g["deg"], Qd, entries_of(g), 10, L_ch, x16=h16 if exact16 else None, ctx=ctx)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt_ = {kn: ctx.kernel_time(kn) for kn in
           ("join", "merge", "init", "sample", "prune", "connect", "search", "exact_knn")}
    ctx.set_timing(False)
    join_ms, join_n, join_work = kt_["join"]

    # search latency: batches of one query (entering points included), then the whole batch
    lat = []
    for i in range(200):
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record()
        pg.search(Xd, g["ids"], g["deg"], Qd[i % Qd.shape[0]:i % Qd.shape[0] + 1], entries, 10, L_ch, x16=x16,
                  ctx=ctx)
        s1.record()
        s1.synchronize()
        lat.append(s0.elapsed_time(s1))
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    pg.search(Xd, g["ids"], g["deg"], Qd, entries, 10, L_ch, x16=x16, ctx=ctx)
    s1.record()
    s1.synchronize()
    qps = Qd.shape[0] / (s0.elapsed_time(s1) / 1000.0)
    ep_lad = ladders["ep"]

    return {
        "_ids": ids, "_graph": g["ids"],
        "points_per_s": n * steps / elapsed,
        "ms_per_step": 1000.0 * elapsed / steps,
        "join_path": st["join_path"], "L": L_ch, "entries": ename,
        "recall@10": rec,
        "recall_ep_only": {"L": ep_lad[-1][0], "recall@10": ep_lad[-1][1]},
        "search_ladders": ladders,
        "knn_recall_sample": knn_recall,
        "knn_d2_rel_error_vs_fp64": d2_err,
        "nndescent_iters": st["iters"], "connect_roots": int(len(g["roots"])),
        "rechecked_fraction": sum(st["rechecked"]) / max(1, sum(st["pairs"])),
        "qps_batch": qps, "search_rows": "fp16 (exact copy)" if exact16 else "fp32",
        "query_latency_ms_batch1": {"p50": float(np.percentile(lat, 50)),
                                    "p99": float(np.percentile(lat, 99))},
        "kernel_ms_per_step": {k: v[0] / steps for k, v in kt_.items()},
        "roofline": roofline(st["join_path"], join_work, join_n, join_ms, path["name"], name),
        "mfma_utilisation": mfma_utilisation(st["join_path"], sum(st["pairs"]) * steps, w["d"], join_ms),
        "bytes_per_build": bytes_per_build(st, w, join_n / steps, path["name"], name),
        "knobs": knobs or "default",
    }


TUNED = True


def tuned_knobs(pg, ctx, Xd, w, prec):
    """The autotuner's cached knobs for this set and precision, or None (the
    library's defaults) when the shape is not in the cache.  The cache key
    names the join path of the default build, taken from one iteration."""
    from paper_2410_01231_amd import tune
    _, _, st = pg.knn_build(Xd, w["K"], S=w["S"], max_iters=1, seed=1, ctx=ctx)
    return tune.lookup(w["n"], w["d"], w["K"], w["S"], st["join_path"], prec, TUNE_CACHE)


def run_tune(args, pg, torch, ctx):
    """Tune the knobs of every set of the suite (or --workload) per join
    precision and write them to --tune-cache."""
    from paper_2410_01231_amd import tune
    names = SUITE if args.workload == "suite" else [args.workload]
    for name in names:
        w = WORKLOADS[name]
        X, _ = gen_data(w)
        Xd = torch.from_numpy(X).cuda()
        del X
        for pname in w["paths"].split(","):
            prec = PATHS[pname]["precision"]
            kn = tune.tune_knn(Xd, w["K"], S=w["S"], seed=1, max_iters=w["iters"], delta=0.001,
                               cache_path=args.tune_cache, ctx=ctx, precision=prec)
            log(f"[bench] tuned {name} {pname}: {kn}")
        del Xd
        torch.cuda.empty_cache()


def bytes_per_build(st, w, join_launches, path_name, workload):
    """The build's compulsory bytes beside the join's HBM traffic measured by
    the counters (per launch, from the profile) times its launches."""
    tr = measured_traffic(path_name, workload)
    return {"compulsory": compulsory_bytes(st, w["n"], w["d"], w["K"], w["S"],
                                           not st["join_path"].startswith("fp32")),
            "join_measured": tr * join_launches if tr is not None else None}


if __name__ == "__main__":
    main()
