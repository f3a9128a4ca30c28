"""Benchmark of the metapath SpGEMM-chain path on one MI355X.

A step evaluates every query of the workload once (scholarly: A-P-V-P-A,
A-P-T-P-A, V-P-T-P-V, T-P-A-P-T on the 4M-author / 6M-paper network, each with
a seeded 1,000-node start set and P.year >= 2015).  The network is resident in
HBM before timing; each query's result stays in device memory (freed after the
query).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scholarly|news]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


# Source regions a kernel's counters depend on: the shared device helpers at
# the top of kernels.hip, the kernel's own section, and internal.hpp.
# sections of kernels.hip a kernel's code lives in (beside the shared helpers at the top)
KERNEL_SECTIONS = {"dense": [("// Visit the flattened products", "// numeric: LDS hash, one wavefront per row"),
                             ("// numeric: dense LDS tiles over column ranges", "// numeric: tile buckets")]}


def kernel_source_digest(kernel: str = "dense") -> str:
    csrc = os.path.join(ROOT, "paper_2201_04058_amd", "csrc")
    with open(os.path.join(csrc, "kernels.hip")) as fh:
        text = fh.read()
    h = hashlib.sha256()
    if kernel == "all":  # every kernel: the whole file
        h.update(text.encode())
    elif kernel in KERNEL_SECTIONS:
        h.update(text[:text.index("// fills, scans")].encode())
        for a, b in KERNEL_SECTIONS[kernel]:
            h.update(text[text.index(a):text.index(b)].encode())
    else:
        h.update(text.encode())
    with open(os.path.join(csrc, "internal.hpp")) as fh:
        hdr = fh.read()
    # constants, enums and argument structs (not the launcher declarations)
    for block in re.findall(r"^(?:constexpr .*?;|enum .*?^};|struct \w+ \{.*?^};)", hdr, re.S | re.M):
        h.update(block.encode())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str, launches_per_step: float) -> float | None:
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_source") != kernel_source_digest(kernel):
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(hin, queries, threads: int, seconds: float) -> dict:
    """The CPU oracle as it stands (its plain left-to-right row chain, OpenMP
    over start rows) timed on the host's cores on a bounded sample: for each
    query a random subset of its start rows, grown by factors of four until it
    takes about seconds / len(queries), timed, and scaled to the whole start
    set (time x |S| / rows) -- an extrapolation, labelled as one."""
    import oracle
    oracle.build(force=False)
    rng = np.random.default_rng(1234)
    budget = seconds / max(1, len(queries))
    est_total, per_query, rows_used, rows_all = 0.0, {}, 0, 0
    for q in queries:
        ids = [c for c in q.constraints if c.kind == "idset" and c.position == 0][0].ids
        k = min(threads, len(ids))
        while True:
            rows = np.sort(rng.choice(ids, size=k, replace=False)).astype(np.int64)
            t0 = time.perf_counter()
            oracle.eval_rows(hin, q, rows, nthreads=threads)
            dt = time.perf_counter() - t0
            if dt >= budget / 4 or k == len(ids):
                break
            k = min(len(ids), k * 4)
        est = dt * len(ids) / k
        est_total += est
        rows_used += k
        rows_all += len(ids)
        per_query[q.name] = {"rows": k, "of": int(len(ids)), "s": round(dt, 3), "est_s_per_query": round(est, 3)}
        log(f"cpu oracle {q.name}: {k} of {len(ids)} start rows in {dt:.2f} s on {threads} threads "
            f"-> {est:.1f} s per query")
    return {"value": len(queries) / est_total, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "extrapolated": rows_used < rows_all,
            "sample": f"per query a random subset of its start rows ({rows_used} of {rows_all} over "
                      f"{len(queries)} queries), timed on {threads} threads and scaled by |start set| / rows; "
                      f"the oracle's left-to-right row chain",
            "per_query": per_query}


# session workloads: entity types that sessions start from, type-level predicates
SESSION_STARTS = {"scholarly": ["A", "V", "T"], "news": ["R", "O", "L"], "tiny": ["A", "T"]}
SESSION_PREDICATES = {"scholarly": {"P": ("year", 2015, 32767)}, "news": {}, "tiny": {}}


def workload_mode(args) -> int:
    """A session workload (Sec. 4.1 "Query Workloads": sessions on one entity,
    restart probability 0.08, metapaths of 3-5 types, shuffled) on the full
    network, evaluated with every cache policy and without a cache."""
    import paper_2201_04058_amd as atp
    from synth import configs, workload

    hin, _ = configs.load(args.workload)
    starts = SESSION_STARTS[args.workload]
    preds = SESSION_PREDICATES[args.workload]
    qs = workload.sessions(hin, 4, args.queries, starts, restart_p=0.08, entities=100, type_predicates=preds)
    stream = None
    try:
        import torch
        torch.cuda.init()
        stream = atp.torch_stream_handle(0)
    except Exception:
        pass
    ctx = atp.Context(device=0, stream=stream)
    ctx.load_hin(hin)
    for q in qs[:20]:  # warm the pool and the planner's statistics
        ctx.eval_query(q).free()
    budget = int(args.cache_gb * (1 << 30))
    rows = {}
    for name in ["OFF", "OTREE", "PGDS", "LRU", "CBS1", "CBS2"]:
        ctx.cache_configure(getattr(atp, "ATP_CACHE_" + name), budget if name != "OFF" else 0)
        lat = []
        t0 = time.perf_counter()
        for q in qs:
            tq = time.perf_counter()
            ctx.eval_query(q).free()
            lat.append(time.perf_counter() - tq)
        el = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        st = ctx.cache_stats()
        rows[name] = {"qps": round(len(qs) / el, 2), "mean_ms": round(float(lat.mean()), 3),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "whole_hits": st["whole_hits"], "sub_hits": st["sub_hits"], "inserts": st["inserts"],
                      "evictions": st["evictions"], "cached_gb": round(st["bytes"] / 2**30, 3)}
        log(f"{name}: {rows[name]}")
    ctx.close()
    out = {"metric": "metapath queries/s (session workload)", "value": rows["OTREE"]["qps"], "unit": "queries/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "int64", "data": "synthetic",
           "config": {"workload": args.workload + "-sessions", "queries": len(qs), "restart_p": 0.08,
                      "cache_gb": args.cache_gb, "start_types": starts},
           "vs_plain_path": round(rows["OTREE"]["qps"] / rows["OFF"]["qps"], 3), "policies": rows}
    print(json.dumps(out), flush=True)
    return 0


def _ctx_with_network(atp, hin):
    stream = None
    try:
        import torch
        torch.cuda.init()
        stream = atp.torch_stream_handle(0)
    except Exception:
        pass
    ctx = atp.Context(device=0, stream=stream)
    ctx.load_hin(hin)
    return ctx


def _pct(a, q):
    return round(float(np.percentile(np.asarray(a), q)), 3) if len(a) else None


def batch_mode(args) -> int:
    """Random schema walks (start type uniform, next type uniform over schema
    neighbours, 3-7 types, a seeded start set, a P-year / D-day window at every
    position of that type), evaluated one at a time and as one batch on lanes
    with fusion.  Both runs produce the same results (the batch tests check
    this); here the result sizes are compared as a guard."""
    import paper_2201_04058_amd as atp
    from synth import configs, workload

    hin, _ = configs.load(args.workload)
    qs = workload.random_walk_batch(hin, 3, args.queries, start_sizes=(args.start_min, args.start_max))
    ctx = _ctx_with_network(atp, hin)
    # the planner's coefficients and the tunables are set before both runs, so
    # that both evaluate the same plans with the same kernels
    tuned = fitted = None
    if args.calibrate:  # Eq. 2 coefficients fitted on walks of another seed
        fitted = ctx.calibrate_cost_model(
            workload.random_walk_batch(hin, 21, args.tune_queries, start_sizes=(args.start_min, args.start_max)))
        log(f"cost model: {fitted}")
    if args.autotune:  # on queries of another seed, not the measured ones
        sample = workload.random_walk_batch(hin, 13, args.tune_queries, start_sizes=(args.start_min, args.start_max))
        tuned = ctx.autotune(sample)
        log(f"autotuned: {tuned}")
    for q in qs[:8]:  # warm-up (a query larger than the device memory fails here as in the runs)
        try:
            ctx.eval_query(q).free()
        except atp.AtpError:
            pass
    t0 = time.perf_counter()
    plain_nnz, lat = [], []
    for z, q in enumerate(qs):
        tq = time.perf_counter()
        try:
            r = ctx.eval_query(q)
            plain_nnz.append(r.shape()[2])
            r.free()
        except atp.AtpError as e:  # e.g. a result larger than the device memory
            plain_nnz.append(("error", e.status))
        lat.append((time.perf_counter() - tq) * 1e3)
        if (z + 1) % args.batch_chunk == 0:
            log(f"  one at a time: {z + 1} of {len(qs)} done, {time.perf_counter() - t0:.1f} s")
    t_plain = time.perf_counter() - t0
    log(f"one at a time: {len(qs)} queries in {t_plain:.2f} s")
    ctx.eval_batch(qs[:8], lanes=args.lanes, max_batch=args.max_batch)
    t0 = time.perf_counter()
    bad, status_diff = [], []
    for c0 in range(0, len(qs), args.batch_chunk):  # batches of batch_chunk queries, one after another
        res = ctx.eval_batch(qs[c0:c0 + args.batch_chunk], lanes=args.lanes, max_batch=args.max_batch,
                             mem_budget_bytes=int(args.admit_gb * (1 << 30)))
        for z, r in enumerate(res, start=c0):
            got = ("error", r.status) if isinstance(r, Exception) else r.shape()[2]
            if got != plain_nnz[z]:
                # a size that differs is a wrong result; a status that differs (one side out of
                # device memory: a batch call holds all its results until it returns) is not
                (status_diff if isinstance(got, tuple) or isinstance(plain_nnz[z], tuple) else bad).append(z)
            if not isinstance(r, Exception):
                r.free()
        log(f"  batch: {min(c0 + args.batch_chunk, len(qs))} of {len(qs)} done, {time.perf_counter() - t0:.1f} s")
    t_batch = time.perf_counter() - t0
    log(f"batch: {len(qs)} queries in {t_batch:.2f} s, mismatches {bad}, status differences {status_diff}")
    ctx.close()
    out = {"metric": "metapath queries/s (batch)", "value": round(len(qs) / t_batch, 3), "unit": "queries/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "int64", "data": "synthetic",
           "config": {"workload": args.workload + "-random-walks", "queries": len(qs), "lengths": [3, 7],
                      "start_set": [args.start_min, args.start_max], "selectivity": [0.01, 0.20],
                      "lanes": args.lanes, "max_batch": args.max_batch, "admit_gb": args.admit_gb,
                      "batch_chunk": args.batch_chunk},
           "one_at_a_time": {"qps": round(len(qs) / t_plain, 3), "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99)},
           "vs_one_at_a_time": round(t_plain / t_batch, 3), "result_mismatches": len(bad),
           "status_differences": len(status_diff), "autotuned": tuned,
           "errors": sorted({int(x[1]) for x in plain_nnz if isinstance(x, tuple)}),
           "n_errors": sum(1 for x in plain_nnz if isinstance(x, tuple)),
           "cost_model": fitted}
    print(json.dumps(out), flush=True)
    return 0 if not bad else 1


def _sampled_rows(r, q, rng, k: int = 12, max_nnz: int = 20_000_000):
    """Up to k start rows of a result (non-empty ones first) with their
    columns and counts, for an oracle check; None for a result too large to
    copy to the host here."""
    n_rows, _, nnz = r.shape()
    if nnz > max_nnz:
        return None
    rp, col, val = r.to_host()
    start = [c for c in q.constraints if c.kind == "idset" and c.position == 0]
    ids = np.asarray(start[0].ids, np.int64) if start else np.arange(n_rows, dtype=np.int64)
    lens = np.diff(rp)
    ne = ids[lens[ids] > 0]
    pick = list(rng.choice(ne, size=min(k - 2, len(ne)), replace=False)) + list(rng.choice(ids, size=min(2, len(ids)),
                                                                                          replace=False))
    rows = np.unique(np.asarray(pick, np.int64))
    return {int(u): (col[rp[u]:rp[u + 1]].copy(), val[rp[u]:rp[u + 1]].copy()) for u in rows}


def _oracle_check(hin, qs, samples) -> dict:
    """Compare the sampled rows of served results with the CPU oracle."""
    import oracle
    oracle.build(force=False)
    bad, rows_checked = [], 0
    for z, got in samples.items():
        if got is None:
            continue
        rows = np.array(sorted(got), np.int64)
        rl, ocol, oval, st = oracle.eval_rows(hin, qs[z], rows, nthreads=max(1, min(len(os.sched_getaffinity(0)), 32)))
        off = np.concatenate([[0], np.cumsum(rl)])
        for i, u in enumerate(rows):
            c, v = got[int(u)]
            if not (np.array_equal(c, ocol[off[i]:off[i + 1]]) and np.array_equal(v, oval[off[i]:off[i + 1]].astype(np.int64))):
                bad.append(int(z))
                break
        rows_checked += len(rows)
    return {"queries_checked": sum(1 for g in samples.values() if g is not None),
            "queries_too_large": sum(1 for g in samples.values() if g is None),
            "rows_checked": rows_checked, "mismatches": len(bad), "mismatch_queries": bad[:8]}


def _serve(atp, ctx, arrivals, qs, lanes, max_batch, admit_bytes, cap_s, check_every: int = 0):
    """Open-loop replay: submit each query at its arrival time, poll
    completions; latency = completion - scheduled arrival.  Every
    check_every-th query's result is sampled for an oracle check."""
    import threading
    ctx.server_start(lanes=lanes, max_batch=max_batch, mem_budget_bytes=admit_bytes)
    n = len(qs)
    done = {}
    t_start = time.perf_counter()
    submitted = [0]

    def feeder():
        for z in range(n):
            wait = arrivals[z] - (time.perf_counter() - t_start)
            if wait > 0:
                time.sleep(wait)
            if time.perf_counter() - t_start > cap_s:
                break
            ctx.submit(qs[z], tag=z)
            submitted[0] = z + 1

    th = threading.Thread(target=feeder)
    th.start()
    next_log = time.perf_counter() + 10
    samples, rng = {}, np.random.default_rng(99)
    while th.is_alive() or len(done) < submitted[0]:
        for cp in ctx.poll(256, wait_ms=50):
            r = cp["result"]
            done[cp["tag"]] = (cp["status"], r.shape()[2] if r is not None else -1, cp["t_done"], cp["batch"])
            if r is not None:
                if check_every and cp["tag"] % check_every == 0:
                    samples[cp["tag"]] = _sampled_rows(r, qs[cp["tag"]], rng)
                r.free()
        if time.perf_counter() > next_log:
            log(f"  {len(done)} of {submitted[0]} submitted done")
            next_log += 10
    th.join()
    wall = time.perf_counter() - t_start
    ctx.server_stop()
    # the server clock starts at server_start, just before t_start
    lat = [(done[z][2] - arrivals[z]) * 1e3 for z in done]
    last = max(d[2] for d in done.values()) if done else 0.0
    return {"completed": len(done), "submitted": submitted[0], "wall_s": round(wall, 3),
            "qps": round(len(done) / max(last, 1e-9), 3),
            "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "mean_ms": round(float(np.mean(lat)), 3),
            "errors": sum(1 for d in done.values() if d[0] != 0),
            "error_status": sorted({int(d[0]) for d in done.values() if d[0] != 0}),
            "error_queries": [qs[z].name for z in sorted(done) if done[z][0] != 0][:8],
            "mean_batch": round(float(np.mean([d[3] for d in done.values()])), 3)}, done, samples


def serve_mode(args) -> int:
    """An open-loop query stream (Poisson arrivals; base walks drawn Zipf(1.0)
    over 500 seeded schema walks of 3-5 types, extended by 0-2-step prefix and
    suffix; start sets and windows from finite seeded pools) served by the
    plain path (one lane, no fusion, no cache) and by the batched + cached
    server (lanes, fusion, Atrapos-OTree cache, slot-memory admission)."""
    import paper_2201_04058_amd as atp
    from synth import configs, workload

    hin, _ = configs.load(args.workload)
    if args.stream == "walks":
        arrivals, qs = workload.serving_stream(hin, 4, args.queries, qps=args.qps,
                                               start_sizes=(args.start_min, args.start_max), pool=args.pool)
    else:  # session queries (one entity each), Poisson arrivals
        qs = workload.sessions(hin, 4, args.queries, SESSION_STARTS[args.workload], restart_p=0.08, entities=100,
                               type_predicates=SESSION_PREDICATES[args.workload])
        gaps = np.random.default_rng(4).exponential(1.0 / args.qps, size=len(qs))
        arrivals = np.cumsum(gaps) - gaps[0]
    ctx = _ctx_with_network(atp, hin)
    # the planner's coefficients and the tunables are set before both paths run
    tuned = fitted = None
    if args.calibrate:  # Eq. 2 coefficients fitted on a stream of another seed
        _, sample = workload.serving_stream(hin, 6, args.tune_queries, start_sizes=(args.start_min, args.start_max),
                                            pool=args.pool)
        fitted = ctx.calibrate_cost_model(sample)
        log(f"cost model: {fitted}")
    if args.autotune:  # on a stream of another seed, not the measured one
        _, sample = workload.serving_stream(hin, 5, args.tune_queries, start_sizes=(args.start_min, args.start_max),
                                            pool=args.pool)
        tuned = ctx.autotune(sample)
        log(f"autotuned: {tuned}")
    for q in qs[:8]:  # warm-up (a query larger than the device memory fails here as in the runs)
        try:
            ctx.eval_query(q).free()
        except atp.AtpError:
            pass
    plain, dp = {"qps": 0.0, "p99_ms": None}, {}
    if not args.no_plain:
        log(f"plain path: {len(qs)} queries at {args.qps} QPS")
        plain, dp, _ = _serve(atp, ctx, arrivals, qs, 1, 1, 0, args.cap_s)
        log(f"plain: {plain}")
    if args.cache_gb > 0:
        ctx.cache_configure(atp.ATP_CACHE_OTREE, int(args.cache_gb * (1 << 30)))
    log(f"served: lanes {args.lanes}, max batch {args.max_batch}, cache {args.cache_gb} GB")
    served, ds, samples = _serve(atp, ctx, arrivals, qs, args.lanes, args.max_batch,
                                 int(args.admit_gb * (1 << 30)), args.cap_s, check_every=args.check_every)
    st = ctx.cache_stats()
    served.update({"whole_hits": st["whole_hits"], "sub_hits": st["sub_hits"], "cache_queries": st["queries"],
                   "hit_rate": round((st["whole_hits"] + st["sub_hits"]) / max(1, st["queries"]), 3),
                   "whole_hit_rate": round(st["whole_hits"] / max(1, st["queries"]), 3)})
    log(f"served: {served}")
    ctx.close()
    # a size that differs is a wrong result; a status that differs (one path out of device memory,
    # e.g. with the cache holding part of it, or under another plan) is not
    both = [z for z in ds if z in dp]
    bad = [z for z in both if ds[z][0] == 0 and dp[z][0] == 0 and ds[z][1] != dp[z][1]]
    status_diff = [z for z in both if (ds[z][0] == 0) != (dp[z][0] == 0)]
    checked = _oracle_check(hin, qs, samples) if samples else None
    log(f"oracle check of served results: {checked}")
    out = {"metric": "metapath queries/s + p50/p99 latency (served stream)", "value": served["qps"],
           "unit": "queries/s", "n_gpus": 1, "higher_is_better": True, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"{args.workload}-{args.stream}-stream", "queries": len(qs), "arrival_qps": args.qps,
                      "start_set": [args.start_min, args.start_max] if args.stream == "walks" else 1,
                      "lanes": args.lanes,
                      "max_batch": args.max_batch, "cache_gb": args.cache_gb, "admit_gb": args.admit_gb,
                      "pool": args.pool},
           "served": served, "plain": plain,
           "vs_plain_qps": round(served["qps"] / max(plain["qps"], 1e-9), 3),
           "vs_plain_p99": round(plain["p99_ms"] / max(served["p99_ms"], 1e-9), 3) if plain["p99_ms"] else None,
           "result_mismatches": len(bad), "status_differences": len(status_diff),
           "status_difference_queries": [qs[z].name for z in status_diff][:8],
           "oracle_check": checked, "autotuned": tuned, "cost_model": fitted}
    print(json.dumps(out), flush=True)
    return 0 if not bad and not (checked and checked["mismatches"]) else 1


def costfit_mode(args) -> int:
    """Planner ablations: the paper's E_ac estimator against the degree-sketch
    estimator, and the Eq. 2 refit -- time every multiplication of a
    calibration sample (random schema walks of another seed), fit alpha,
    beta, gamma, delta, and compare plans and times of the workload's queries
    and of a held-out sample under the default and the fitted coefficients."""
    import paper_2201_04058_amd as atp
    from synth import configs, workload

    hin, queries = configs.load(args.workload)
    calib = workload.random_walk_batch(hin, 21, args.tune_queries, start_sizes=(args.start_min, args.start_max))
    held = workload.random_walk_batch(hin, 22, args.queries, start_sizes=(args.start_min, args.start_max))
    ctx = _ctx_with_network(atp, hin)

    def run(qs, reps=3):
        for q in qs:
            ctx.eval_query(q).free()
        best, plans = None, []
        for _ in range(reps):
            t0 = time.perf_counter()
            plans = []
            for q in qs:
                r = ctx.eval_query(q)
                plans.append(r.stats()["plan"])
                r.free()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best * 1e3, plans

    default = ctx.cost_model()
    ctx.set_flags(plan_eac=True)  # the paper's uniform E_ac estimator (Sec. 3.2)
    we, wpe = run(queries)
    he, hpe = run(held, reps=1)
    ctx.set_flags()
    w0, wp0 = run(queries)
    h0, hp0 = run(held, reps=1)
    fit = ctx.calibrate_cost_model(calib)
    log(f"fit: {fit}")
    w1, wp1 = run(queries)
    h1, hp1 = run(held, reps=1)
    ctx.close()
    out = {"metric": "planned workload time (ms), default vs fitted Eq. 2 coefficients", "unit": "ms",
           "n_gpus": 1, "dtype": "int64", "data": "synthetic",
           "config": {"workload": args.workload, "calibration_queries": len(calib), "held_out_queries": len(held),
                      "start_set": [args.start_min, args.start_max]},
           "default_coeffs": default, "fitted": fit,
           "workload_ms": {"default": round(w0, 3), "fitted": round(w1, 3)},
           "workload_plans": {q.name: [a, b] for q, a, b in zip(queries, wp0, wp1)},
           "held_out_ms": {"default": round(h0, 3), "fitted": round(h1, 3)},
           "held_out_plans_changed": sum(1 for a, b in zip(hp0, hp1) if a != b),
           "estimators": {"eac": {"workload_ms": round(we, 3), "held_out_ms": round(he, 3),
                                  "workload_plans": {q.name: p for q, p in zip(queries, wpe)}},
                          "sketch": {"workload_ms": round(w0, 3), "held_out_ms": round(h0, 3)}}}
    print(json.dumps(out), flush=True)
    return 0


def _pmc_per_kernel(db: str) -> dict:
    """kernel name -> (sum of the counter over its dispatches in KiB, dispatches)
    from a rocprofv3 --pmc database holding one counter."""
    import sqlite3
    con = sqlite3.connect(db)
    agg = {}
    for name, value, did in con.execute("select name, counter_value, dispatch_id from pmc_events"):
        a = agg.setdefault(name, [0.0, set()])
        a[0] += value
        a[1].add(did)
    con.close()
    return {k: (v[0], len(v[1])) for k, v in agg.items()}


# kernels of the counting pass only (bench.py's untimed byte count), and the
# runtime's copy kernels (network upload, small read-backs): not part of a step
COUNTING_KERNELS = ("k_bin_stats", "k_mark_bytes")


def counters_summary(args) -> int:
    """profiles/traffic_dense_<w>.json (the dominant kernel) and
    profiles/traffic_chain_<w>.json (every kernel of a step) from FETCH_SIZE /
    WRITE_SIZE databases of `bench.py --workload <w> --steps 1 --warmup 0
    --no-side-by-side --no-cpu-baseline --no-news` (each query evaluated in four
    passes: shapes, byte count, serial profile, timed step) and of the copy
    calibration, whose counters give the KiB-to-bytes scale."""
    fdb, wdb, cfdb, cwdb = args.counters_summary
    w = args.workload
    copy_bytes = 1024 << 20

    def copy_scale(db):
        pk = _pmc_per_kernel(db)
        name = max(pk, key=lambda k: pk[k][0] / pk[k][1])  # the 1 GiB copy dominates
        per = pk[name][0] / pk[name][1]
        return copy_bytes / (per * 1024.0), per

    fscale, fcopy = copy_scale(cfdb)
    wscale, wcopy = copy_scale(cwdb)
    fk, wk = _pmc_per_kernel(fdb), _pmc_per_kernel(wdb)
    passes = 4
    rows, total = [], 0.0
    for name in sorted(set(fk) | set(wk)):
        if any(x in name for x in COUNTING_KERNELS) or name.startswith("__amd_rocclr"):
            continue
        f, nf = fk.get(name, (0.0, 0))
        wv, nw = wk.get(name, (0.0, 0))
        b = (f * fscale + wv * wscale) * 1024.0 / passes
        total += b
        rows.append((b, name, nf // passes, f / max(nf, 1), wv / max(nw, 1)))
    rows.sort(reverse=True)
    cmd = {"fetch": f"HSA_ENABLE_SDMA=0 rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_FETCH_SIZE_{w} -o run -- python3 bench.py --workload {w} "
                    "--steps 1 --warmup 0 --no-side-by-side --no-cpu-baseline --no-news",
           "write": f"HSA_ENABLE_SDMA=0 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_WRITE_SIZE_{w} -o run -- python3 bench.py --workload {w} "
                    "--steps 1 --warmup 0 --no-side-by-side --no-cpu-baseline --no-news",
           "copy_fetch": "HSA_ENABLE_SDMA=0 rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_copy_FETCH_SIZE -o run -- python3 bench.py "
                         "--copy-calibration 1024",
           "copy_write": "HSA_ENABLE_SDMA=0 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_copy_WRITE_SIZE -o run -- python3 bench.py "
                         "--copy-calibration 1024",
           "summary": "python3 bench.py --workload W --counters-summary FETCH.db WRITE.db COPY_FETCH.db COPY_WRITE.db"}
    calib = (f"a 1 GiB device-to-device copy: FETCH_SIZE {fcopy:.1f} KiB -> scale {fscale:.4f}, "
             f"WRITE_SIZE {wcopy:.1f} KiB -> scale {wscale:.4f}")
    chain = {"workload": w, "kernel_source": kernel_source_digest("all"), "bytes_per_step": round(total),
             "passes": passes, "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
             "calibration": calib, "commands": cmd,
             "per_kernel": [{"kernel": n, "bytes_per_step": round(b), "dispatches_per_step": d,
                             "fetch_kib_per_dispatch": round(f, 1), "write_kib_per_dispatch": round(x, 1)}
                            for b, n, d, f, x in rows]}
    with open(os.path.join(ROOT, "profiles", f"traffic_chain_{w}.json"), "w") as fh:
        json.dump(chain, fh, indent=1)
    dn = [n for n in fk if "k_dense(" in n]
    if dn:
        f, nf = fk[dn[0]]
        wv, nw = wk.get(dn[0], (0.0, 1))
        dense = {"kernel": "dense", "workload": w, "kernel_source": kernel_source_digest("dense"),
                 "fetch_kib_per_dispatch": round(f / nf, 1), "write_kib_per_dispatch": round(wv / nw, 1),
                 "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4), "dispatches": nf,
                 "bytes_per_launch": round((f / nf * fscale + wv / nw * wscale) * 1024.0),
                 "calibration": calib, "commands": cmd}
        with open(os.path.join(ROOT, "profiles", f"traffic_dense_{w}.json"), "w") as fh:
            json.dump(dense, fh, indent=1)
        dl = [f"# HBM traffic of k_dense on workload {w} (rocprofv3 --pmc, one counter per run)",
              f"# fetch: {cmd['fetch']}", f"# write: {cmd['write']}",
              f"# copy calibration: {cmd['copy_fetch']} ; {cmd['copy_write']}", calib,
              f"k_dense: {nf} dispatches, FETCH_SIZE {f / nf:.1f} KiB/dispatch, WRITE_SIZE {wv / nw:.1f} KiB/dispatch",
              f"scaled HBM traffic per dispatch: {dense['bytes_per_launch'] / 1e6:.1f} MB"]
        with open(os.path.join(ROOT, "profiles", f"traffic_dense_{w}.txt"), "w") as fh:
            fh.write("\n".join(dl) + "\n")
    lines = [f"# HBM traffic per step, workload {w} (rocprofv3 --pmc, one counter per run)",
             f"# fetch: {cmd['fetch']}", f"# write: {cmd['write']}",
             f"# copy calibration: {cmd['copy_fetch']} ; {cmd['copy_write']}",
             f"{calib}", f"every kernel of a step (4 passes per run, counting kernels and runtime copies excluded): "
             f"{total / 1e6:.1f} MB per step", "",
             f"{'kernel':60s} {'disp/step':>9s} {'MB/step':>9s} {'fetch KiB/disp':>15s} {'write KiB/disp':>15s}"]
    for b, n, d, f, x in rows[:16]:
        lines.append(f"{n[:60]:60s} {d:9d} {b / 1e6:9.1f} {f:15.1f} {x:15.1f}")
    with open(os.path.join(ROOT, "profiles", f"traffic_chain_{w}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines), flush=True)
    return 0


def probe_mode(args) -> int:
    """Each query of the workload once, the bins of every product serialised:
    under `rocprofv3 --pmc` the k_dense dispatches then come in the order
    this prints ({"query", "product"} per dispatch, one JSON line), so that
    `--dense-counters` can label them."""
    os.environ["ATP_PROFILE_STEPS"] = "1"  # kernel names carry the product's index
    import paper_2201_04058_amd as atp
    from synth import configs
    hin, queries = configs.load(args.workload)
    ctx = _ctx_with_network(atp, hin)
    order = []
    for q in queries:
        ctx.set_flags(profile=True, serial_bins=True)
        ctx.kernel_times_reset()
        ctx.eval_query(q).free()
        names = [k for k, v in ctx.kernel_times().items() if k.startswith("dense#") and v[1] > 0]
        for k in sorted(names, key=lambda x: int(x.split("#")[1])):
            order.append({"query": q.name, "product": int(k.split("#")[1])})
    ctx.set_flags()
    ctx.close()
    print(json.dumps({"workload": args.workload, "dense_dispatches": order}), flush=True)
    return 0


DENSE_COUNTER_GROUPS = (
    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_ACTIVE_INST_VALU "
    "SQ_INSTS_VALU",
    "SQ_INSTS_LDS SQ_ACTIVE_INST_LDS SQ_LDS_BANK_CONFLICT SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_WAIT_INST_LDS "
    "TCC_HIT_sum TCC_MISS_sum")


def dense_counters(args) -> int:
    """profiles/counters_dense_<workload>.txt: every k_dense dispatch of
    `bench.py --probe` runs under rocprofv3 --pmc (one database per counter
    group), labelled with the probe's query and product."""
    probe_json, dbs = args.dense_counters[0], args.dense_counters[1:]
    with open(probe_json) as fh:
        probe = json.loads(fh.read().strip().splitlines()[-1])
    labels = probe["dense_dispatches"]
    w = probe["workload"]
    import sqlite3
    per = {}  # label index -> counter -> value
    durs = {}
    for db in dbs:
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, name, counter_name, counter_value, duration from pmc_events").fetchall()
        con.close()
        disp = {}
        for did, name, cn, cv, du in rows:
            if "k_dense(" not in name:
                continue
            disp.setdefault(did, {}).setdefault(cn, 0.0)
            disp[did][cn] += cv
            disp[did]["_dur"] = du
        ids = sorted(disp)
        if len(ids) != len(labels):
            raise SystemExit(f"{db}: {len(ids)} k_dense dispatches, the probe lists {len(labels)}")
        for i, did in enumerate(ids):
            durs.setdefault(i, []).append(disp[did].pop("_dur") / 1e3)
            per.setdefault(i, {}).update(disp[did])
    lines = [f"# k_dense counters on workload {w}, one k_dense dispatch per row (rocprofv3 --pmc, one group per run)",
             f"# probe: python3 bench.py --workload {w} --probe > gpurun_out/probe_{w}.json"]
    for z, g in enumerate(DENSE_COUNTER_GROUPS):
        lines.append(f"# group {z + 1}: timeout -s KILL 120 rocprofv3 --pmc {g} -d gpurun_out/pmc_dense{z + 1}_{w} -o run "
                     f"-- python3 bench.py --workload {w} --probe")
    lines.append(f"# summary: python3 bench.py --dense-counters gpurun_out/probe_{w}.json "
                 + " ".join(f"gpurun_out/pmc_dense{z + 1}_{w}/run_results.db" for z in range(len(DENSE_COUNTER_GROUPS))))
    lines.append("# SQ_* counts are summed over the device; *_CYCLES and SQ_WAIT_* / SQ_ACTIVE_* are wave-cycles of the")
    lines.append("# sequencers (in the same unit, so their ratios hold); TCC_* are L2 requests")
    lines.append("")
    cols = ["dur_us", "waves", "valu/wave", "salu/wave", "vmem/wave", "lds/wave", "wait_any", "wait_inst", "valu_busy",
            "lds_bank", "L2_hit"]
    lines.append(f"{'query':24s} {'prod':>4s} " + " ".join(f"{c:>10s}" for c in cols))
    for i, lab in enumerate(labels):
        c = per.get(i, {})
        wv = max(c.get("SQ_WAVES", 0.0), 1.0)
        wc = max(c.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        hit, miss = c.get("TCC_HIT_sum", 0.0), c.get("TCC_MISS_sum", 0.0)
        vals = [sum(durs.get(i, [0])) / max(len(durs.get(i, [])), 1), c.get("SQ_WAVES", 0.0),
                c.get("SQ_INSTS_VALU", 0.0) / wv, c.get("SQ_INSTS_SALU", 0.0) / wv, c.get("SQ_INSTS_VMEM_RD", 0.0) / wv,
                c.get("SQ_INSTS_LDS", 0.0) / wv, c.get("SQ_WAIT_ANY", 0.0) / wc, c.get("SQ_WAIT_INST_ANY", 0.0) / wc,
                c.get("SQ_ACTIVE_INST_VALU", 0.0) / wc,
                c.get("SQ_LDS_BANK_CONFLICT", 0.0) / max(c.get("SQ_ACTIVE_INST_LDS", 0.0), 1.0),
                hit / max(hit + miss, 1.0)]
        lines.append(f"{lab['query']:24s} {lab['product']:4d} " + " ".join(f"{v:10.3f}" if v < 100 else f"{v:10.0f}"
                                                                        for v in vals))
    lines += ["", "wait_any, wait_inst, valu_busy: SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_ACTIVE_INST_VALU over SQ_WAVE_CYCLES "
              "(share of a wave's life); lds_bank: SQ_LDS_BANK_CONFLICT over SQ_ACTIVE_INST_LDS; L2_hit: TCC hits over "
              "hits + misses; per-wave columns: instructions per wave"]
    with open(os.path.join(ROOT, "profiles", f"counters_dense_{w}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines), flush=True)
    return 0


# numeric kernels whose algorithmic bytes make up a product's compulsory bytes
# (operands read once, result written once); the compaction copy and the
# scans are design overhead
NUMERIC_KERNELS = ("hash_wave", "hash_block", "dense", "bucket")


def host_info() -> dict:
    """The host the CPU baseline ran on: logical CPUs, the ones this process
    may use, and the CPU model from lscpu (or /proc/cpuinfo)."""
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in txt.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info["lscpu_" + k.strip().lower().replace("(s)", "s").replace(" ", "_")] = v.strip()
    except Exception:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    info["model_name"] = ln.split(":", 1)[1].strip()
                    break
    return info


def chain_traffic(workload: str) -> dict | None:
    """Counter (FETCH_SIZE + WRITE_SIZE) bytes of every kernel of one step,
    from the committed summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_chain_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_source") != kernel_source_digest("all"):
        return None
    return t


def plain_record(atp, configs, args, workload: str, side_by_side: bool, cpu: bool) -> dict:
    """One workload's queries evaluated one at a time: the JSON record."""
    t0 = time.perf_counter()
    hin, queries = configs.load(workload)
    log(f"workload {workload}: {len(queries)} queries, network ready in {time.perf_counter() - t0:.1f} s")
    stream = None
    try:
        import torch
        torch.cuda.init()
        stream = atp.torch_stream_handle(0)
    except Exception:
        torch = None
    ctx = atp.Context(device=0, stream=stream, plan_eac=args.plan_eac)
    ctx.load_hin(hin)
    log(f"network registered: {ctx.device_bytes() / 2**30:.2f} GiB on the device")

    # plans and shapes (one untimed pass, also warms the pool)
    plans = {}
    for q in queries:
        r = ctx.eval_query(q)
        plans[q.name] = r.stats()
        r.free()
        log(f"  {q.name}: {plans[q.name]}")

    # algorithmic bytes per kernel, per query and per step (counting mode, untimed)
    ctx.set_flags(count_bytes=True, plan_eac=args.plan_eac)
    bytes_per_step, comp_per_query = {}, {}
    for q in queries:
        ctx.kernel_times_reset()
        ctx.eval_query(q).free()
        kb = {k: v[2] for k, v in ctx.kernel_times().items()}
        for k, v in kb.items():
            bytes_per_step[k] = bytes_per_step.get(k, 0.0) + v
        comp_per_query[q.name] = sum(kb.get(k, 0.0) for k in NUMERIC_KERNELS)
    ctx.set_flags(plan_eac=args.plan_eac)

    # dominant kernel: the most device time in one pass with a product's bins
    # on one stream (in the timed region they run side by side, so their event
    # spans would overlap); the per-kernel table comes from this pass
    ctx.set_flags(profile=True, serial_bins=True, plan_eac=args.plan_eac)
    ctx.kernel_times_reset()
    for q in queries:
        ctx.eval_query(q).free()
    serial = {k: v for k, v in ctx.kernel_times().items() if v[1] > 0}
    ctx.set_flags(plan_eac=args.plan_eac)
    dom = max(serial, key=lambda k: serial[k][0])

    for _ in range(args.warmup):
        for q in queries:
            ctx.eval_query(q).free()

    # timed region: HIP events around the dominant kernel's launches only (on
    # the stream each runs on); every other launch runs unprofiled
    ctx.set_profile_kernel(dom)
    ctx.set_flags(profile=True, plan_eac=args.plan_eac)
    ctx.kernel_times_reset()
    lat = []
    if stream is not None:
        torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        for q in queries:
            tq = time.perf_counter()
            r = ctx.eval_query(q)
            lat.append(time.perf_counter() - tq)
            r.free()
    if stream is not None:
        torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    kt = ctx.kernel_times()
    ctx.set_flags(plan_eac=args.plan_eac)
    ctx.set_profile_kernel(None)
    n_q = len(queries) * args.steps
    qps = n_q / elapsed
    lat_ms = np.array(lat) * 1e3
    ms_per_step = elapsed / args.steps * 1e3

    # the same steps with each step's queries side by side on four lanes (the
    # engine's batch call; the queries differ, so nothing is fused); every
    # result's nnz is checked against the one-at-a-time pass
    conc_lanes = 4

    def conc_step():
        for q, r in zip(queries, ctx.eval_batch(queries, lanes=conc_lanes, max_batch=1)):
            if isinstance(r, atp.AtpError):
                raise r
            if r.shape()[2] != plans[q.name]["nnz"]:
                raise RuntimeError(f"{q.name}: {r.shape()[2]} nonzeros side by side, {plans[q.name]['nnz']} alone")
            r.free()
    conc_elapsed = None
    if side_by_side:
        for _ in range(max(1, args.warmup)):
            conc_step()
        if stream is not None:
            torch.cuda.synchronize()
        t_c = time.perf_counter()
        for _ in range(args.steps):
            conc_step()
        if stream is not None:
            torch.cuda.synchronize()
        conc_elapsed = time.perf_counter() - t_c

    ms_total, launches, _ = kt[dom]
    alg_bytes = bytes_per_step.get(dom, 0.0) * args.steps
    achieved = alg_bytes / (ms_total * 1e-3) / 1e9 if ms_total > 0 else 0.0
    launches_per_step = launches / args.steps
    traffic = traffic_for(dom, workload, launches_per_step)
    # per kernel, from the serialised pass (one step): device ms, launches, algorithmic GB/s
    per_kernel = {k: {"serial_ms_per_step": round(v[0], 4), "launches_per_step": v[1],
                      "alg_GBps": round(bytes_per_step.get(k, 0.0) / (v[0] * 1e-3) / 1e9, 1)
                      if v[0] > 0 and bytes_per_step.get(k) else None}
                  for k, v in sorted(serial.items(), key=lambda kv: -kv[1][0])}
    per_kernel[dom]["timed_ms_per_step"] = round(ms_total / args.steps, 4)

    # the whole chain: compulsory bytes of every product (operands read once,
    # result written once, restricted to the rows launched) over the query's
    # time, and the counters' HBM bytes of every kernel of the step
    comp_step = sum(comp_per_query.values())
    med = {q.name: float(np.median(lat_ms[i::len(queries)])) for i, q in enumerate(queries)}
    chain = {"compulsory_bytes_per_step": round(comp_step),
             "compulsory_GBps": round(comp_step / (ms_per_step * 1e-3) / 1e9, 1),
             "frac": round(comp_step / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "per_query": {q.name: {"compulsory_bytes": round(comp_per_query[q.name]),
                                    "median_ms": round(med[q.name], 3),
                                    "compulsory_GBps": round(comp_per_query[q.name] / (med[q.name] * 1e-3) / 1e9, 1)}
                           for q in queries}}
    ct = chain_traffic(workload)
    if ct:
        cb = ct["bytes_per_step"]
        chain.update({"counter_bytes_per_step": round(cb), "counter_GBps": round(cb / (ms_per_step * 1e-3) / 1e9, 1),
                      "counter_frac": round(cb / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    else:
        chain.update({"counter_bytes_per_step": None, "counter_GBps": None, "counter_frac": None})
    start = [c for c in queries[0].constraints if c.kind == "idset" and c.position == 0]

    out = {
        "metric": "metapath queries/s",
        "value": round(qps, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "queries": [q.name for q in queries],
                   "start_set": int(len(start[0].ids)) if start else None,
                   "network": {t: int(n) for t, n in hin.counts.items()},
                   "edges": int(sum(r.nnz for r in hin.relations.values())),
                   "parallelism": "single-gpu"},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "per_query_median": {k: round(v, 3) for k, v in med.items()}},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "alg_bytes_per_launch": round(alg_bytes / launches, 1) if launches else None,
                     "avg_launch_ms": round(ms_total / launches, 5) if launches else None,
                     # HBM traffic (counters) over the same launch time, and its share of peak
                     "traffic_GBps": round(traffic / (ms_total / launches * 1e-3) / 1e9, 1)
                     if traffic and launches else None,
                     "traffic_frac": round(traffic / (ms_total / launches * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                     if traffic and launches else None},
        "chain": chain,
        "kernels": per_kernel,
        "serial_kernel_ms_per_step": round(sum(v[0] for v in serial.values()), 3),
        "launches_per_query": round(sum(v[1] for v in serial.values()) / len(queries), 1),
        "plans": {k: v["plan"] for k, v in plans.items()},
        "n_op_per_step": int(sum(v["n_op"] for v in plans.values())),
        "products_per_s": round(sum(v["n_op"] for v in plans.values()) / (elapsed / args.steps), 1),
        "nnz_result_per_step": int(sum(v["nnz"] for v in plans.values())),
        # not the headline: the queries of a step evaluated concurrently instead of one at a time
        "side_by_side": {"lanes": conc_lanes, "queries_per_s": round(n_q / conc_elapsed, 3),
                         "ms_per_step": round(conc_elapsed / args.steps * 1e3, 3)} if conc_elapsed else None,
    }
    ctx.close()
    if cpu:
        threads = max(1, min(len(os.sched_getaffinity(0)), 64))
        out["cpu_baseline"] = cpu_baseline(hin, queries, threads, args.cpu_seconds)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="scholarly", choices=["scholarly", "news", "tiny"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU oracle baseline: about this many seconds of sampled work per workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-news", action="store_true", help="scholarly: skip the news sub-record")
    ap.add_argument("--counters-summary", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="write profiles/traffic_*_<workload>.json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE "
                         "databases of `bench.py --steps 1 --warmup 0 --no-side-by-side --no-cpu-baseline "
                         "--no-news` and of `bench.py --copy-calibration 1024`")
    ap.add_argument("--probe", action="store_true",
                    help="each query once, bins serialised; prints the order of the k_dense dispatches")
    ap.add_argument("--dense-counters", nargs="+", metavar="PATH",
                    help="PROBE_JSON DB...: write profiles/counters_dense_<workload>.txt from rocprofv3 --pmc "
                         "databases of `bench.py --probe`")
    ap.add_argument("--no-side-by-side", action="store_true",
                    help="skip the second timed region (the step's queries side by side on four lanes)")
    ap.add_argument("--plan-eac", action="store_true", help="paper's uniform E_ac planner")
    ap.add_argument("--mode", default="plain", choices=["plain", "workload", "batch", "serve", "costfit"],
                    help="plain: the workload's queries, one at a time; workload: a session query stream "
                         "evaluated with each cache policy (Sec. 3.3-3.4) against the plain path; batch: random "
                         "walks one at a time and as a batch; serve: an open-loop stream, plain path and server")
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--admit-gb", type=float, default=64.0, help="batch/serve: slot-memory admission budget")
    ap.add_argument("--start-min", type=int, default=100)
    ap.add_argument("--start-max", type=int, default=5000)
    ap.add_argument("--qps", type=float, default=200.0, help="serve: arrival rate")
    ap.add_argument("--cap-s", type=float, default=120.0, help="serve: stop submitting after this many seconds")
    ap.add_argument("--pool", type=int, default=16, help="serve: start sets per type and windows in the pools")
    ap.add_argument("--autotune", action="store_true", help="batch/serve: autotune the tunables first")
    ap.add_argument("--calibrate", action="store_true", help="batch/serve: refit Eq. 2's coefficients first")
    ap.add_argument("--tune-queries", type=int, default=24)
    ap.add_argument("--no-plain", action="store_true", help="serve: skip the plain-path run")
    ap.add_argument("--check-every", type=int, default=10,
                    help="serve: sample rows of every n-th served result and compare them with the CPU oracle")
    ap.add_argument("--batch-chunk", type=int, default=16,
                    help="batch: queries per eval_batch call (a call holds all its results until it returns)")
    ap.add_argument("--stream", default="walks", choices=["walks", "sessions"],
                    help="serve: extended schema walks with pooled constraints, or session queries")
    ap.add_argument("--queries", type=int, default=500, help="workload/batch/serve: queries")
    ap.add_argument("--cache-gb", type=float, default=4.0, help="workload/serve: cache budget")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    if args.copy_calibration:
        # three device-to-device copies of a known size through the HIP runtime
        import ctypes
        rt = ctypes.CDLL("libamdhip64.so.7")
        rt.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        rt.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
        rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        rt.hipFree.argtypes = [ctypes.c_void_p]
        n = args.copy_calibration << 20
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        if rt.hipMalloc(ctypes.byref(a), n) or rt.hipMalloc(ctypes.byref(b), n) or rt.hipMemset(a, 1, n):
            raise RuntimeError("copy calibration: device allocation failed")
        for _ in range(3):
            if rt.hipMemcpy(b, a, n, 3):  # device to device
                raise RuntimeError("copy calibration: copy failed")
        rt.hipDeviceSynchronize()
        rt.hipFree(a)
        rt.hipFree(b)
        print(json.dumps({"copy_bytes": n}), flush=True)
        return 0

    import paper_2201_04058_amd as atp
    from synth import configs

    if args.mode == "workload":
        return workload_mode(args)
    if args.mode == "batch":
        return batch_mode(args)
    if args.mode == "serve":
        return serve_mode(args)
    if args.mode == "costfit":
        return costfit_mode(args)

    if args.dense_counters:
        return dense_counters(args)
    if args.probe:
        return probe_mode(args)
    if args.counters_summary:
        return counters_summary(args)

    out = plain_record(atp, configs, args, args.workload, side_by_side=not args.no_side_by_side,
                       cpu=not args.no_cpu_baseline)
    if args.workload == "scholarly" and not args.no_news:
        # the news workload (its own network and queries), measured the same way
        news = plain_record(atp, configs, args, "news", side_by_side=False, cpu=not args.no_cpu_baseline)
        out["news"] = {k: news[k] for k in ("metric", "value", "unit", "ms_per_step", "config", "latency_ms",
                                            "roofline", "chain", "plans", "n_op_per_step", "products_per_s",
                                            "nnz_result_per_step", "launches_per_query", "cpu_baseline")
                       if k in news}
    out["host"] = host_info()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
