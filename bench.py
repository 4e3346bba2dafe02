"""Benchmark: one 300-residue query against the 500,200-target synthetic
database (log-normal lengths, median 300), the full search path per step:
pair scoring, device ranking (top 500) and alignments of the top 50.
`--workload batched` measures instead 256 queries of U[30, 1000] residues
against the 2,020-target database as one batch (one persistent scoring launch,
replayed from a captured graph), beside the same 256 queries searched one at
a time; `--workload long` does the same for 32 queries of U[2000, 5000]
residues against that database plus 5,064 targets of 10,000-35,000 residues.
`--workload serving` replays Poisson query arrivals at 50, 200 and 500 queries/s
(lengths log-normal, median 250) into the serving loop over the 2,020-target
database and reports p50/p99 latency and the sustained rate.  `--workload sw`
times the Smith-Waterman-Gotoh scores of the full workload's query against
every target beside the heuristic's search of the same query (its roofline
counts 11 32-bit integer ops per cell against 256 CUs x 64 lanes x 2.4 GHz =
39.3 TOP/s).

The default run also measures the rest of the metric in the same line: a
`batched` object (the 256-query batch against the same queries searched one
at a time, with the batch scoring kernel's roofline) and a `serving` object
(p50/p99 latency and the sustained rate at 50, 200 and 500 queries/s, plus a
saturating 5,000 queries/s for information).

Prints one JSON line.  `value` is query*database residues per second with the
database and the query resident in device memory when timing starts.  The
roofline object covers the dominant kernel (pair scoring): algorithmic integer
ops (2 per scored residue pair -- one substitution-score fetch, one add) per
launch divided by its mean duration, timed with HIP events on its own stream.
The peak is the vector ALU's byte-operation rate, 256 CUs x 64 lanes x 4 bytes
per 32-bit op x 2.4 GHz = 157.3 TOP/s: the kernel does its adds four bytes to a
32-bit op, and the same figure in cells (78.6 T/s) is the rate at which LDS
delivers one score byte per cell at 128 bytes per clock per CU.  cpu_baseline
times the single-threaded oracle on a bounded, deterministic sample of the
same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 4 byte lanes per 32-bit op, 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 4 * 2.4e9 / 1e12
OPS_PER_CELL = 2


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


SCORING_SOURCES = ("device_common.hpp", "score_kernels.hpp")


def _launch_text(src):
    """The part of hs_lib.hip that sizes and launches the one-query scoring
    kernel: from query_layout through the end of launch_score (with the
    constants between them)."""
    i = src.index("\nint query_layout(")
    j = src.index("\n}\n", src.index("\nint launch_score(", i))
    return src[i:j + 3]


def kernel_source_hash():
    """Hash of the sources the scoring kernel and its launch are built from:
    the device code and the host code that sizes and launches it."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1508_06561_amd", "csrc")
    for f in SCORING_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(_launch_text(open(os.path.join(csrc, "hs_lib.hip")).read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch of the scoring kernel from the committed
    rocprofv3 counter summary, or None when the kernel sources changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", "score_full_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def host_facts():
    """Host CPU facts for the CPU baseline: logical CPUs (nproc), the CPUs
    this process may run on, and the model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(w, q, budget_s):
    """Oracle (plain single-threaded C) on every m-th target, m chosen so the
    sample takes about budget_s seconds."""
    import numpy as np
    import oracle as O
    codes = O.encode_db(w.residues, w.offsets)
    qc = O.encode(bytes(q))
    # calibrate on a small stride
    probe = np.arange(0, w.n_targets, 997, dtype=np.int64)
    t = time.perf_counter()
    O.score_all(codes, w.offsets, qc, O.Params(), ids=probe)
    dt = max(time.perf_counter() - t, 1e-3)
    m = max(1, int(w.n_targets / (len(probe) * budget_s / dt)))
    ids = np.arange(0, w.n_targets, m, dtype=np.int64)
    t = time.perf_counter()
    O.score_all(codes, w.offsets, qc, O.Params(), ids=ids)
    dt = time.perf_counter() - t
    res = int(np.diff(w.offsets)[ids].sum())
    return {"value": len(q) * res / dt, "unit": "query*residues/s", "cores": 1, "kind": "oracle",
            "sample": f"every {m}th target ({len(ids)} of {w.n_targets}, {res} residues), "
                      f"one query of {len(q)}, single thread, {dt:.1f} s", **host_facts()}


def cpu_baseline_batched(w, budget_s, stride=1):
    """Oracle on the first m queries of the batch against every stride-th
    target, m chosen so that the sample takes about budget_s seconds."""
    import numpy as np
    import oracle as O
    codes = O.encode_db(w.residues, w.offsets)
    ids = np.arange(0, w.n_targets, stride, dtype=np.int64)
    tres = int(np.diff(w.offsets)[ids].sum())
    t = time.perf_counter()
    m, res = 0, 0
    while m < len(w.queries) and time.perf_counter() - t < budget_s:
        O.score_all(codes, w.offsets, O.encode(bytes(w.queries[m])), O.Params(),
                    ids=ids if stride > 1 else None)
        res += len(w.queries[m]) * tres
        m += 1
    dt = time.perf_counter() - t
    which = f"every {stride}th target ({len(ids)} of {w.n_targets})" if stride > 1 else \
        f"all {w.n_targets} targets"
    return {"value": res / dt, "unit": "query*residues/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} of {len(w.queries)} queries against {which}, "
                      f"single thread, {dt:.1f} s", **host_facts()}


BATCH_WORKLOADS = {
    "batched": dict(gen="config_batched", metric="batch of 256 queries",
                    desc="256 queries U[30,1000] vs 2,020 targets U[50,500] (20 planted homologs); "
                         "top 50 ranked and aligned per query; one persistent scoring launch, "
                         "graph replay",
                    data="synthetic (seeded; uniform query lengths, background residue composition)",
                    cpu_stride=1),
    "long": dict(gen="config_long", metric="batch of 32 long queries",
                 desc="32 queries U[2000,5000] vs 2,020 targets U[50,500] plus 5,064 targets "
                      "U[10000,35000] (64 planted homologs); top 50 ranked and aligned per query; "
                      "one persistent scoring launch, graph replay",
                 data="synthetic (seeded; uniform lengths, background residue composition)",
                 cpu_stride=64),
}


def bench_batched(args):
    out = measure_batched(args, args.workload)
    print(json.dumps(out), flush=True)


def measure_batched(args, workload, cpu=True):
    import numpy as np
    import torch

    import paper_1508_06561_amd as H
    import synth

    spec = BATCH_WORKLOADS[workload]
    w = getattr(synth, spec["gen"])()
    qs = [bytes(q) for q in w.queries]
    nres = sum(map(len, qs))
    log(f"{workload} workload: {len(qs)} queries ({nres} residues) vs {w.n_targets} targets, "
        f"{w.db_residues} residues")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    db = H.Database(w.residues, w.offsets)
    p = H.Params()
    b = H.Batch(db, len(qs), max(map(len, qs)), nres, k=w.k, n_aln=w.n_aln)
    b.set(qs, p)
    log(f"default schedule {b.get_schedule()}")
    if args.schedule:
        b.schedule(*args.schedule)
        sched = b.get_schedule()
        log(f"fixed schedule {sched}")
    else:
        tuned_ms = b.tune(reps=3 if workload == "batched" else 1)
        sched = b.get_schedule()
        log(f"tuned schedule {sched}: scoring {tuned_ms:.3f} ms")
    sched["launch"] = b.get_launch()
    for _ in range(args.warmup):
        b.run(graph=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        b.run(graph=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"batch of {len(qs)}: {ms:.3f} ms per batch (graph replay)")
    ev0.record(stream)
    for _ in range(args.steps):
        b.run(graph=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_eager = ev0.elapsed_time(ev1) / args.steps
    log(f"batch of {len(qs)}: {ms_eager:.3f} ms per batch (direct launches)")

    # dominant kernel alone: the batch scoring pass, with its cell count
    cells_t = torch.zeros(1, dtype=torch.int64, device="cuda")
    b.score(cells_t)
    torch.cuda.synchronize()
    cells = int(cells_t.cpu()[0])
    ev0.record(stream)
    for _ in range(args.steps):
        b.score()
    ev1.record(stream)
    torch.cuda.synchronize()
    k_ms = ev0.elapsed_time(ev1) / args.steps
    achieved = cells * OPS_PER_CELL / (k_ms * 1e-3) / 1e12
    log(f"batch scoring kernel: {k_ms:.3f} ms, {cells} cells, "
        f"{cells / (k_ms * 1e-3) / 1e12:.3f} Tcells/s")

    # the same queries one at a time (hs_search_dev, same database)
    codes = np.concatenate([H.encode(q) for q in qs])
    offs = np.zeros(len(qs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(q) for q in qs])
    d_codes = torch.from_numpy(codes).cuda()
    ds = H.DeviceSearch(db, max(map(len, qs)), w.k, w.n_aln)

    def one_by_one():
        for i in range(len(qs)):
            db.search_dev(d_codes[offs[i]:offs[i + 1]], len(qs[i]), p, w.k, w.n_aln, ds.ws,
                          ds.hits, ds.n_hits, ds.alns, ds.ops, ds.stride)
    one_by_one()
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    ev0.record(stream)
    for _ in range(reps):
        one_by_one()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_single = ev0.elapsed_time(ev1) / reps
    log(f"one at a time: {ms_single:.3f} ms for {len(qs)} queries")

    recall = None
    # Setting a batch builds its round-0 draw table (one Philox pass over the
    # database) when the seed differs from the cached table's; the replays
    # above reuse the cached table, while each one-at-a-time search runs its
    # own draw kernel.  Timed here with a fresh seed on every set (host
    # encode, upload and table), for a like-for-like ratio.
    reps_set = max(1, args.steps // 4)
    t_set = 0.0
    for i in range(reps_set):
        pf = H.Params(seed=1000 + i)
        torch.cuda.synchronize()
        t = time.perf_counter()
        b.set(qs, pf)
        b.run(graph=False)
        torch.cuda.synchronize()
        t_set += time.perf_counter() - t
    ms_set_run = t_set * 1e3 / reps_set
    b.set(qs, p)
    log(f"set (fresh seed) + run: {ms_set_run:.3f} ms per batch")

    if workload == "long":
        # two planted homologs per query, in query order
        hits = b.results()
        per = len(w.planted) // len(qs)
        found = sum(int(t) in set(int(x) for x in hits[i].hits["target_id"])
                    for i in range(len(qs)) for t in w.planted[per * i:per * (i + 1)])
        recall = {"k": w.k, "planted": len(w.planted), "recall": found / len(w.planted),
                  "note": "each query's planted homologs ranked in its top k (information only)"}

    qres = nres * w.db_residues
    out = {
        "metric": f"query*DB residues/sec on 1 GPU ({spec['metric']})",
        "value": qres / (ms * 1e-3),
        "unit": "query*residues/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": spec["data"],
        "config": {"workload": spec["desc"],
                   "query_residues": nres, "db_residues": w.db_residues, "k": w.k,
                   "n_aln": w.n_aln, "schedule": sched,
                   "params": "PGP 0, GOP 10, GEP 5, LFactor 0.5, SFactor 1, MinFactor 0.5, "
                             "Rounds 1"},
        "ms_direct_launch": ms_eager,
        "one_at_a_time": {"ms": ms_single, "value": qres / (ms_single * 1e-3),
                          "batch_speedup": ms_single / ms},
        "draw_table": {"note": "hs_batch_set caches the round-0 random-draw table per "
                               "(database, seed); graph replays reuse it, each one-at-a-time "
                               "search runs its own draw kernel",
                       "ms_set_fresh_seed_and_run": ms_set_run,
                       "batch_speedup_incl_set": ms_single / ms_set_run},
        "roofline": {"bound": "alu", "kernel": "k_score_batch", "achieved": achieved,
                     "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS,
                     "traffic": None, "ops_per_cell": OPS_PER_CELL,
                     "cells_per_launch": cells, "kernel_ms": k_ms,
                     "cells_per_s": cells / (k_ms * 1e-3)},
    }
    if recall is not None:
        out["homolog_recall"] = recall
    if cpu and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batched(w, args.cpu_budget, spec["cpu_stride"])
        log(f"cpu baseline: {out['cpu_baseline']}")
    b.close()
    db.close()
    return out


def bench_serving(args):
    rows = measure_serving(args, args.rates)
    top = rows[-1]
    out = {
        "metric": f"p99 query latency (serving, Poisson {top['rate']} queries/s)",
        "value": top["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": sum(r["queries"] for r in rows),
        "warmup": 16,
        "ms_per_step": top["mean_ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded; Poisson arrivals, log-normal query lengths)",
        "config": {"workload": SERVING_DESC.format(rates=", ".join(f"{r:g}" for r in args.rates),
                                                   secs=args.serve_s)},
        "serving": rows,
    }
    print(json.dumps(out), flush=True)


SERVING_DESC = ("Poisson arrivals at {rates} queries/s for {secs} s each, |Q| log-normal (median "
                "250, sigma 0.6, clip 20-2,000), vs 2,020 targets U[50,500]; top 500 hits and "
                "top 50 alignments per query; continuous batching (at most 64 queries per "
                "batch, two batches in flight)")


def measure_serving(args, rates):
    import threading

    import numpy as np
    import torch

    import paper_1508_06561_amd as H
    import synth

    torch.cuda.set_device(0)
    w0 = synth.config_serving(50, duration_s=0.1)
    db = H.Database(w0.residues, w0.offsets)
    srv = H.Server(db, max_batch=64, max_qlen=2000, max_residues=64 * 2000, k=w0.k, n_aln=w0.n_aln,
                   workers=2)
    # warm-up: first launches and allocations
    for i, q in enumerate(w0.queries[:16]):
        srv.submit(bytes(q), tag=(1 << 40) + i)
    got = 0
    while got < min(16, len(w0.queries)):
        for t in srv.poll(timeout_ms=100):
            srv.result(t)
            got += 1
    # and queries one at a time, so that one-query batches' paths run too
    for i, q in enumerate(w0.queries[:8]):
        srv.submit(bytes(q), tag=(1 << 41) + i)
        done = False
        while not done:
            for t in srv.poll(timeout_ms=100):
                srv.result(t)
                done = True
    rows = []
    for ri, rate in enumerate(rates):
        w = synth.config_serving(rate, duration_s=args.serve_s)
        qs = [bytes(q) for q in w.queries]
        base = (ri + 1) << 32
        t0 = time.perf_counter()

        def feed():
            for i, ta in enumerate(w.arrivals):
                d = t0 + float(ta) - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                srv.submit(qs[i], tag=base + i)

        th = threading.Thread(target=feed)
        th.start()
        timings = []
        while len(timings) < len(qs):
            for t in srv.poll(timeout_ms=200):
                _, tm = srv.result(t)
                tm["qlen"] = len(qs[t - base])
                timings.append(tm)
        th.join()
        lat = np.array([t["total_ms"] for t in timings])
        slow = sorted(range(len(timings)), key=lambda i: -timings[i]["total_ms"])[:3]
        qms = np.array([t["queue_ms"] for t in timings])
        bms = np.array([t["batch_ms"] for t in timings])
        start = min(t["submit_ms"] for t in timings)
        end = max(t["submit_ms"] + t["total_ms"] for t in timings)
        row = {"rate": rate, "queries": len(qs), "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
               "mean_ms": float(lat.mean()),
               "p99_queue_ms": float(np.percentile(qms, 99)),
               "p99_batch_ms": float(np.percentile(bms, 99)),
               "sustained_qps": len(qs) / ((end - start) * 1e-3),
               "mean_batch": float(np.mean([t["batch_size"] for t in timings])),
               "max_batch": int(max(t["batch_size"] for t in timings)),
               "mean_batch_ms": float(bms.mean()),
               "slowest": [{"total_ms": timings[i]["total_ms"], "queue_ms": timings[i]["queue_ms"],
                            "batch_ms": timings[i]["batch_ms"], "set_ms": timings[i]["set_ms"],
                            "run_ms": timings[i]["run_ms"], "results_ms": timings[i]["results_ms"],
                            "gpu_ms": timings[i]["gpu_ms"],
                            "batch_size": timings[i]["batch_size"], "qlen": timings[i]["qlen"],
                            "at_s": (timings[i]["submit_ms"] - start) * 1e-3} for i in slow]}
        log(f"rate {rate}/s: {row}")
        rows.append(row)
    srv.close()
    db.close()
    return rows


def measure_threshold(args, db, ds, w):
    """Threshold reporting (every target at or above min_score, ranked, no
    cap) on the full workload's query: a threshold admitting about 100,000
    targets and none (all 500,200 ranked), device form, HIP events."""
    import numpy as np
    import torch

    import paper_1508_06561_amd as H

    stream = torch.cuda.current_stream()
    scores = torch.empty(w.n_targets, dtype=torch.int32, device="cuda")
    db.score_dev(ds.q, ds.qlen, H.Params(), ds.ws, scores)
    s = np.sort(scores.cpu().numpy())[::-1]
    ws = torch.empty(db.threshold_workspace_bytes(), dtype=torch.uint8, device="cuda")
    hits = torch.empty(w.n_targets * 16, dtype=torch.uint8, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    rows = []
    for label, thr in (("about 100,000 targets", int(s[100_000])), ("every target", -(2**31))):
        p = H.Params(min_score=thr)
        for _ in range(2):
            db.search_threshold_dev(ds.q, ds.qlen, p, w.n_targets, 0, ws, hits, n)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            db.search_threshold_dev(ds.q, ds.qlen, p, w.n_targets, 0, ws, hits, n)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        rows.append({"threshold": label, "min_score": thr, "hits": int(n.cpu()[0]),
                     "ms_per_search": ms})
        log(f"threshold search ({label}): {ms:.3f} ms, {int(n.cpu()[0])} hits")
    return {"workload": "the full workload's query, every target at or above min_score ranked "
                        "(no cap), device form", "rows": rows}


def measure_align(args):
    """Pairwise mode (every overlapping placement, best of Rounds = 20) on
    1,000 pairs: a log-normal query (median 300) against a mutated copy with
    indels (20-90% identity) embedded in a flank, plus the longest accepted
    pair (5,600 x 5,600); host in and out (hs_align_batch)."""
    import numpy as np
    import torch

    import paper_1508_06561_amd as H
    import synth

    rng = np.random.default_rng(synth.BASE_SEED + 7)
    pairs = []
    for L in synth.lognormal_lengths(rng, 1000, 300, 0.6, 20, 2000):
        q = synth.random_protein(rng, int(L))
        tl = int(synth.lognormal_lengths(rng, 1, 300, 0.6, 20, 2000)[0])
        t = synth.embed(rng, synth.mutate(rng, q, rng.uniform(0.2, 0.9)), tl)[:5600]
        pairs.append((bytes(q), bytes(t)))
    p = H.Params(rounds=20)
    H.align_batch(pairs, p)          # the first call of this size grows the allocation pool
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = max(3, args.steps // 5)
    for _ in range(reps):
        H.align_batch(pairs, p)
    ms = (time.perf_counter() - t) * 1e3 / reps
    # the same pairs with the letters resident in device memory and the
    # results left there (hs_align_batch_dev): HIP events around the calls
    qs = [H.encode(q) for q, _ in pairs]
    ts = [H.encode(t) for _, t in pairs]
    qoff = np.cumsum([0] + [len(q) for q in qs])
    toff = np.cumsum([0] + [len(t) for t in ts]) + qoff[-1]
    d_codes = torch.from_numpy(np.concatenate(qs + ts)).cuda()
    n = len(pairs)
    d_ws = torch.empty(H.align_workspace_bytes(n, 20), dtype=torch.uint8, device="cuda")
    d_sc = torch.empty(n, dtype=torch.int32, device="cuda")
    d_rd = torch.empty(n, dtype=torch.int32, device="cuda")
    d_ops = torch.empty(int(toff[-1]), dtype=torch.int32, device="cuda")
    d_nops = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def dev():
        H.align_batch_dev(d_codes, qoff, toff, p, d_ws, d_sc, d_rd, d_ops, d_nops)
    dev()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        dev()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_dev = ev0.elapsed_time(ev1) / reps
    big = (bytes(synth.random_protein(rng, 5600)), bytes(synth.random_protein(rng, 5600)))
    H.align(*big, p)
    t = time.perf_counter()
    H.align(*big, p)
    ms_big = (time.perf_counter() - t) * 1e3
    log(f"pairwise mode: {ms:.2f} ms per 1,000 pairs (Rounds 20; {ms_dev:.2f} ms device-resident), "
        f"longest pair {ms_big:.2f} ms")
    out = {"workload": "pairwise mode (Fig. 1 full slide), Rounds 20: 1,000 pairs, query "
                       "log-normal median 300, target a 20-90% identity copy with indels in a "
                       "flank; host in and out",
           "ms_per_1000_pairs": ms, "pairs_per_s": 1000 / (ms * 1e-3),
           "ms_per_1000_pairs_device_resident": ms_dev,
           "pairs_per_s_device_resident": 1000 / (ms_dev * 1e-3),
           "ms_longest_pair_5600x5600": ms_big}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_align(pairs, args.cpu_budget / 4)
        log(f"cpu baseline (pairwise mode): {out['cpu_baseline']}")
    return out


def cpu_baseline_align(pairs, budget_s):
    """Oracle pairwise mode (plain single-threaded C, Rounds 20, full slide)
    on the benchmark's pairs in order until about budget_s seconds have
    passed."""
    import oracle as O
    op = O.Params(rounds=20, full_slide=True)
    n = 0
    t = time.perf_counter()
    while n < len(pairs) and time.perf_counter() - t < budget_s:
        q, tg = pairs[n]
        O.align_pair(O.encode(q), O.encode(tg), target_id=n, params=op)
        n += 1
    dt = time.perf_counter() - t
    return {"value": n / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {len(pairs)} pairs, Rounds 20, single thread, {dt:.1f} s",
            **host_facts()}


SW_OPS_PER_CELL = 11     # Gotoh cell: 4 subtractions, 1 addition, 6 maxima (with the running best)
SW_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit integer ops: 64 lanes per CU per clock


def cpu_baseline_sw(w, q, budget_s):
    """Oracle Gotoh checker (plain single-threaded C) on targets in index
    order until about budget_s seconds have passed."""
    import numpy as np
    import oracle as O
    codes = O.encode_db(w.residues, w.offsets)
    qc = O.encode(bytes(q))
    res = 0
    n = 0
    t = time.perf_counter()
    while n < w.n_targets and time.perf_counter() - t < budget_s:
        O.sw_score(qc, codes[w.offsets[n]:w.offsets[n + 1]])
        res += int(w.offsets[n + 1] - w.offsets[n])
        n += 1
    dt = time.perf_counter() - t
    return {"value": len(q) * res / dt, "unit": "query*residues/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {w.n_targets} targets ({res} residues), one query of "
                      f"{len(q)}, single thread, {dt:.1f} s", **host_facts()}


def bench_sw(args):
    """Smith-Waterman-Gotoh scores of the full workload's query against every
    target (hs_sw_scores_dev), beside the heuristic's whole search of the
    same query: the speed and sensitivity comparison of Sections I and IV."""
    import numpy as np
    import torch

    import paper_1508_06561_amd as H
    import synth

    w = synth.config_full()
    q = w.queries[0]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    db = H.Database(w.residues, w.offsets)
    p = H.Params()
    ds = H.DeviceSearch(db, len(q), w.k, w.n_aln)
    ds.set_query(bytes(q))
    scores = torch.empty(w.n_targets, dtype=torch.int32, device="cuda")
    ws = torch.empty(db.sw_workspace_bytes(), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        db.sw_scores_dev(ds.q, ds.qlen, p, ws, scores)
        ds.run(p)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        db.sw_scores_dev(ds.q, ds.qlen, p, ws, scores)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    ev0.record(stream)
    for _ in range(args.steps):
        ds.run(p)
    ev1.record(stream)
    torch.cuda.synchronize()
    h_ms = ev0.elapsed_time(ev1) / args.steps
    res = ds.fetch()
    log(f"sw scores: {ms:.3f} ms; heuristic search: {h_ms:.3f} ms")
    sw = scores.cpu().numpy()
    ids = np.arange(w.n_targets)
    top_sw = ids[np.lexsort((ids, -sw.astype(np.int64)))][:w.k]
    planted = set(int(x) for x in w.planted)
    recall_sw = len(planted & set(int(x) for x in top_sw)) / len(planted)
    recall_h = len(planted & set(int(x) for x in res.hits["target_id"])) / len(planted)
    cells = len(q) * w.db_residues
    achieved = cells * SW_OPS_PER_CELL / (ms * 1e-3) / 1e12
    out = {
        "metric": "query*DB residues/sec on 1 GPU (one query, Smith-Waterman-Gotoh scores)",
        "value": cells / (ms * 1e-3),
        "unit": "query*residues/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded; log-normal lengths, background residue composition)",
        "config": {"workload": "one 300-residue query vs 500,200 targets (log-normal lengths, "
                               "median 300, sigma 0.6, clip 10-35,000; 200 planted homologs); "
                               "every target's optimal local score",
                   "db_residues": w.db_residues, "params": "GOP 10, GEP 5, BLOSUM62"},
        "roofline": {"bound": "alu", "kernel": "k_sw_scores", "achieved": achieved,
                     "peak": SW_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / SW_PEAK_TOPS,
                     "traffic": None, "ops_per_cell": SW_OPS_PER_CELL, "cells_per_launch": cells,
                     "kernel_ms": ms, "cells_per_s": cells / (ms * 1e-3)},
        "heuristic": {"ms_per_search": h_ms, "sw_over_heuristic_time": ms / h_ms},
        "homolog_recall": {"k": w.k, "planted": len(planted), "sw": recall_sw,
                           "heuristic": recall_h,
                           "note": "planted homologs ranked in the top k (information only)"},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_sw(w, q, args.cpu_budget)
        log(f"cpu baseline: {out['cpu_baseline']}")
    db.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["full", "batched", "long", "serving", "sw", "align"],
                    default="full")
    ap.add_argument("--letters", type=int, choices=[8, 5], default=8,
                    help="full workload: letter image of the scoring kernel (8 = bytes, 5 = packed)")
    ap.add_argument("--rates", type=float, nargs="+", default=[50, 200, 500])
    ap.add_argument("--schedule", type=int, nargs=3, metavar=("COPIES", "CAP", "CHUNK"),
                    help="batch workloads: fixed schedule instead of the autotuner")
    ap.add_argument("--serve-s", type=float, default=2.0, help="seconds of arrivals per rate")
    ap.add_argument("--saturate", type=float, default=5000.0,
                    help="default run: an extra serving rate beyond the three of the workload "
                         "(0: none)")
    ap.add_argument("--full-only", action="store_true",
                    help="default run: the one-query line alone, without the batched and "
                         "serving objects")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the search shards by target range across GPUs "
              "by design, but this build measures the single-GPU kernel (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload in BATCH_WORKLOADS:
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "sw":
        return bench_sw(args)
    if args.workload == "align":
        print(json.dumps(measure_align(args)), flush=True)
        return

    import numpy as np
    import torch

    import paper_1508_06561_amd as H
    import synth

    t0 = time.perf_counter()
    w = synth.config_full()
    q = w.queries[0]
    log(f"workload generated in {time.perf_counter() - t0:.1f}s: {w.n_targets} targets, "
        f"{w.db_residues} residues")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    db = H.Database(w.residues, w.offsets)
    if args.letters != 8:
        db.set_letters(args.letters)
    torch.cuda.synchronize()
    log(f"database loaded: {db.info()}, letters {args.letters} bits")
    p = H.Params()
    ds = H.DeviceSearch(db, len(q), w.k, w.n_aln)
    ds.set_query(bytes(q))

    for _ in range(args.warmup):
        ds.run(p)
    torch.cuda.synchronize()
    log("warmup done")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        ds.run(p)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    res = ds.fetch()
    log(f"timed {args.steps} steps: {ms:.3f} ms/step, {len(res.hits)} hits")
    top = set(int(x) for x in res.hits["target_id"])
    recall = sum(int(x) in top for x in w.planted) / len(w.planted)

    # dominant kernel alone (pair scoring), same stream, HIP events
    scores = torch.empty(w.n_targets, dtype=torch.int32, device="cuda")
    cells_t = torch.zeros(1, dtype=torch.int64, device="cuda")
    db.score_dev(ds.q, ds.qlen, p, ds.ws, scores, None, cells_t)
    torch.cuda.synchronize()
    cells = int(cells_t.cpu()[0])
    ev0.record(stream)
    for _ in range(args.steps):
        db.score_dev(ds.q, ds.qlen, p, ds.ws, scores)
    ev1.record(stream)
    torch.cuda.synchronize()
    k_ms = ev0.elapsed_time(ev1) / args.steps
    achieved = cells * OPS_PER_CELL / (k_ms * 1e-3) / 1e12
    log(f"scoring kernel: {k_ms:.3f} ms, {cells} cells, {cells / (k_ms * 1e-3) / 1e12:.3f} Tcells/s")

    qres = len(q) * w.db_residues
    out = {
        "metric": "query*DB residues/sec on 1 GPU, batched vs one-query; p50/p99 query latency",
        "value": qres / (ms * 1e-3),
        "unit": "query*residues/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded; log-normal lengths, background residue composition)",
        "config": {"workload": "one 300-residue query vs 500,200 targets (log-normal lengths, "
                               "median 300, sigma 0.6, clip 10-35,000; 200 planted homologs); "
                               "top 500 ranked, top 50 aligned",
                   "db_residues": w.db_residues, "k": w.k, "n_aln": w.n_aln,
                   "params": "PGP 0, GOP 10, GEP 5, LFactor 0.5, SFactor 1, MinFactor 0.5, "
                             "Rounds 1"},
        "roofline": {"bound": "alu", "kernel": "k_score_sched", "achieved": achieved,
                     "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS,
                     "traffic": traffic_from_profile(), "ops_per_cell": OPS_PER_CELL,
                     "cells_per_launch": cells, "kernel_ms": k_ms,
                     "cells_per_s": cells / (k_ms * 1e-3)},
    }
    out["homolog_recall"] = {"k": w.k, "planted": len(w.planted), "recall": recall,
                             "note": "planted homologs ranked in the top k (information only)"}
    if args.letters != 8:
        out["config"]["letters"] = f"{args.letters}-bit image"
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, q, args.cpu_budget)
        log(f"cpu baseline: {out['cpu_baseline']}")
    if not args.full_only:
        out["threshold"] = measure_threshold(args, db, ds, w)
    db.close()
    del ds, scores, cells_t
    if not args.full_only:
        # the rest of the metric: the batched search against the one-query
        # kernel, and serving latency, as objects of the same line
        bt = measure_batched(args, "batched", cpu=False)
        out["batched"] = {"workload": bt["config"]["workload"], "value": bt["value"],
                          "unit": bt["unit"], "ms_per_batch": bt["ms_per_step"],
                          "ms_direct_launch": bt["ms_direct_launch"],
                          "one_at_a_time": bt["one_at_a_time"], "draw_table": bt["draw_table"],
                          "schedule": bt["config"]["schedule"], "roofline": bt["roofline"]}
        rates = list(args.rates) + ([args.saturate] if args.saturate else [])
        rows = measure_serving(args, rates)
        out["align"] = measure_align(args)
        out["serving"] = {"workload": SERVING_DESC.format(rates=", ".join(f"{r:g}" for r in rates),
                                                          secs=args.serve_s),
                          "rows": rows,
                          "note": f"{args.saturate:g} q/s is a saturating rate, information only"
                                  if args.saturate else ""}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
