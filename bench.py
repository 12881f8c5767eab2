"""Benchmark: connected 4-vertex subgraphs counted per second on one MI355X.

Default workload (the configuration the metric names first): a batch of 4096 directed
G(n, p) graphs, n ~ U{20..500}, mean out-degree ~ U[2, 8], counted for k = 4 by one
batched launch (whole-graph kernel, replayed from a captured HIP graph, launch
parameters from the autotuner) against 4096 per-graph launches on the same GPU.  One
step = one batched launch over all 4096 graphs, inputs resident in HBM.  The same JSON
line carries the serving run (Poisson arrivals, continuous batching, p50/p99) and the
oracle timed on the host cores.

Other workloads (``--workload``): ``chunglu`` (n = 1e6 Chung-Lu, k = 3 and 4 in one
call), ``rmat22`` (R-MAT scale 22, k = 4), ``er1000``, ``chunglu_u`` (undirected
motifs), ``serve`` (the serving workload alone at its full pool).  There, one step =
device graph build + one count call.

Every count is checked: column sums are multiples of k and equal k x the number of sets
the kernels visited one by one (the per-shape visit counters); batched = per-graph,
served = alone.  Bit-exact parity with the oracle is the test suite's job.

Prints ONE JSON line.  ``--gpus N`` with N > 1 exits with a message: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                       # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12    # 32-bit VALU lane-ops/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
MODEL_OPS_PER_SET = 40                      # per-set integer work of the method, k = 3, 4 (lower end)
MODEL_OPS_PER_SET5 = 60                     # k = 5: 20-bit index, 4 pair tests, lookup, 5 credits

WORKLOADS = {
    "batch4096": "4096 directed G(n,p) graphs, n ~ U{20..500}, mean out-degree ~ U[2,8], graph i seeded (3,i); "
                 "k=4 in one batched launch (autotuned, HIP-graph replay) vs 4096 per-graph launches",
    "chunglu": "Chung-Lu directed power-law graph, n=1,000,000, 8.4M base arcs (~10M arcs), "
               "gamma 2.1, undirected degree cap 2000, 20% reciprocated, seed 2; k=3 and k=4 in one call",
    "er1000": "directed G(n=1000, p=0.005), seed 1; k=3 and k=4 in one call",
    "rmat22": "R-MAT scale 22, edge factor 8, (0.57,0.19,0.19,0.05), cap 1500, seed 4; k=4",
    "chunglu_u": "the Chung-Lu graph with arc directions ignored; undirected 4-vertex motifs (6 classes)",
    "serve": "serving: pool of resident ER and Chung-Lu graphs (even/odd), n log-uniform, mean out-degree "
             "U[2,10], k in {3,4} 50/50, Poisson arrivals at 0.5x and 0.8x the measured capacity",
    "chunglu5000_k5": "5-vertex motifs of one Chung-Lu graph too large for LDS (n = 5000, the chunglu recipe "
                      "scaled down: ~50k arcs, max degree 141), counted in device memory",
    "batch256_k5": "5-vertex motifs (9364 classes): the first 256 graphs of the batch4096 recipe (directed "
                   "G(n,p), n ~ U{20..500}, mean out-degree ~ U[2,8], graph i seeded (3,i)); one batched "
                   "launch (graphs cut into parts by estimated work) vs 256 per-graph launches",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# ---------------------------------------------------------------------------------------------
# counters from committed rocprofv3 runs (profiles/), keyed by a hash of the kernel sources

_CS = "paper_2201_11655_amd/csrc/"
# kernel sources behind each workload's counters: a change to any of them voids the
# committed counters of that workload
COUNTER_SOURCES = {
    "batch4096": [_CS + "small.hip", _CS + "count.hip", _CS + "batch.hip", _CS + "motif_device.h",
                  _CS + "vdmc_internal.h"],
    "chunglu": [_CS + "count.hip", _CS + "count_hub.hip", _CS + "motif_device.h", _CS + "vdmc_internal.h"],
    "batch256_k5": [_CS + "count5.hip", _CS + "vdmc_internal.h"],
    "chunglu5000_k5": [_CS + "count5.hip", _CS + "motif_device.h", _CS + "vdmc_internal.h"],
}
COUNTER_SOURCES["rmat22"] = COUNTER_SOURCES["chunglu"]
COUNTER_SOURCES["chunglu_u"] = COUNTER_SOURCES["chunglu"]
COUNTER_SOURCES["er1000"] = COUNTER_SOURCES["chunglu"]
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0   # FETCH_SIZE / WRITE_SIZE of a 1 GiB copy read 0.5x / 1.0x its bytes


def sources_sha256(workload):
    h = hashlib.sha256()
    for f in COUNTER_SOURCES.get(workload, []):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_counters(workload):
    """Per-launch counters of the dominant kernel(s) from profiles/counters.json, or None when
    they were taken with other kernel sources."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("sources_sha256") != sources_sha256(workload):
        return None
    return rec


def roofline(workload, sets, kernel_ms, kernel_name, compulsory_bytes, ops_per_set=MODEL_OPS_PER_SET):
    """ALU roofline of the dominant kernel(s).  achieved = the method's per-set work (ops_per_set
    32-bit lane-ops: index assembly, edge tests, class lookup, k credits) x the sets one launch
    visits, over the launch time measured live; peak = the VALU lane-op rate of the chip.
    From the committed counters of the same kernel sources (profiles/counters.json): the HBM
    traffic per launch (FETCH_SIZE x 2 + WRITE_SIZE, the copy-calibrated factors), the issued
    VALU lane-ops, and the memory-side atomics."""
    secs = kernel_ms * 1e-3
    achieved = ops_per_set * sets / secs / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
           "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "kernel": kernel_name, "kernel_ms": kernel_ms,
           "sets_per_launch": sets, "ops_per_set": ops_per_set,
           "hbm_compulsory_bytes": compulsory_bytes,
           "hbm_compulsory_frac": compulsory_bytes / secs / 1e9 / HBM_PEAK_GBS}
    rec = load_counters(workload)
    if rec is None:
        out["note"] = "no committed counters for these kernel sources: traffic unmeasured"
        return out
    traffic = 1024.0 * (FETCH_FACTOR * rec["fetch_kib"] + WRITE_FACTOR * rec["write_kib"])
    out["traffic"] = traffic
    out["traffic_frac_of_hbm"] = traffic / secs / 1e9 / HBM_PEAK_GBS
    lane_ops = 64.0 * rec["valu_insts"]
    out["measured"] = {
        "valu_lane_ops_per_s": lane_ops / secs / 1e12, "valu_frac": lane_ops / secs / 1e12 / VALU_PEAK_TOPS,
        "valu_lane_slots_per_set": lane_ops / max(sets, 1),
        "memory_side_atomics": rec["tcc_ea0_atomic"], "atomics_per_s": rec["tcc_ea0_atomic"] / secs,
        "counter_kernel_ms": rec.get("trace_ms"),
    }
    return out


# ---------------------------------------------------------------------------------------------
# the oracle on the host cores

def cpu_baseline_batch(graphs, budget_s):
    """The oracle (as it is) on the batch workload: all 4096 graphs on every host core, and
    on one core over the first graphs until about budget_s/2 of work; plus the small ER
    graph er1000 in full."""
    import graphgen as gg
    import oracle
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    sets_all = 0
    for g in graphs:
        _, tot = oracle.count(g.n, g.src, g.dst, 4, threads=threads)
        sets_all += int(tot.sum())
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    sets_one, done = 0, 0
    for g in graphs:
        _, tot = oracle.count(g.n, g.src, g.dst, 4, threads=1)
        sets_one += int(tot.sum())
        done += 1
        if time.perf_counter() - t0 > budget_s / 2:
            break
    t_one = time.perf_counter() - t0
    e = gg.config_graph("er1000")
    t0 = time.perf_counter()
    _, tot = oracle.count(e.n, e.src, e.dst, 4, threads=threads)
    t_er = time.perf_counter() - t0
    return {
        "value": sets_all / t_all, "unit": "4-vertex sets/s", "cores": threads, "kind": "oracle",
        "sample": f"oracle ESU + k!-canonicalisation, full count of all {len(graphs)} graphs ({sets_all} sets) "
                  f"in {t_all:.1f} s on {threads} threads",
        "one_core": {"value": sets_one / t_one, "graphs": done, "sets": sets_one, "seconds": t_one},
        "er1000": {"value": int(tot.sum()) / t_er, "sets": int(tot.sum()), "seconds": t_er, "cores": threads},
        "cpu_model": cpu_model(), "nproc": os.cpu_count(),
    }


def cpu_baseline_rows(g, budget_s, k=4):
    """Large graphs: the oracle's per-vertex mode on seeded random vertices of the graph
    until about budget_s of work, as (vertex, set) incidences per second; a full count is
    out of reach on the host (extrapolation = sets / rate)."""
    import oracle
    rng = np.random.default_rng(12345)
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    cand = np.flatnonzero(deg > 0)
    threads = oracle.default_threads()
    rows, sets, used = 0, 0, 0.0
    while used < budget_s and rows < cand.size:
        pick = rng.choice(cand, size=threads, replace=False).astype(np.int32)
        t0 = time.perf_counter()
        out = oracle.count_rows(g.n, g.src, g.dst, k, pick, threads=threads)
        used += time.perf_counter() - t0
        sets += int(out.sum())
        rows += threads
    return {"value": sets / used if used > 0 else None, "unit": f"(vertex, {k}-set) incidences/s", "cores": threads,
            "kind": "oracle", "sample": f"oracle per-vertex mode on {rows} seeded random non-isolated vertices: "
                                        f"{sets} incidences in {used:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


# ---------------------------------------------------------------------------------------------

def visited_sets(v, G, k):
    sc = v.shape_counts(G)
    return sc["(1,1)"] + sc["(1,2)"] if k == 3 else sc["(3,0,0)"] + sc["(2,1,0)"] + sc["(1,2,0)"] + sc["(1,1,1)"]


def bench_batch(args, torch, gg, v):
    t0 = time.perf_counter()
    graphs = gg.er_batch(4096, 20, 500, 2.0, 8.0, seed=3)
    log(f"[bench] generated 4096 graphs ({sum(g.n for g in graphs)} vertices) in {time.perf_counter() - t0:.1f}s")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    outs = [torch.empty((g.n, 199), dtype=torch.int64, device="cuda") for g in graphs]
    t0 = time.perf_counter()
    choice = v.tuned_choice(Gs, 4)
    if not choice.get("tuned"):   # no choice for this batch shape in VDMC_TUNE_CACHE: tune now
        v.tune(Gs, 4, args.tune_cache)
        choice = v.tuned_choice(Gs, 4)
    log(f"[bench] tuned in {time.perf_counter() - t0:.1f}s: {choice}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for w in range(args.warmup):
            v.count_batch(Gs, 4, outs=outs, stream=stream)
            stream.synchronize()
            log(f"[bench] warmup {w} done")
        v.count_batch(Gs, 4, outs=outs, stream=stream)   # at least one capture before timing
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            v.count_batch(Gs, 4, outs=outs, stream=stream)
        ev1.record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        ms_batch = (time.perf_counter() - t0) * 1e3 / args.steps
        dev_ms = ev0.elapsed_time(ev1) / args.steps
        log(f"[bench] {args.steps} batched steps: {ms_batch:.3f} ms/step (device {dev_ms:.3f} ms)")
        col = sum(o.sum(dim=0) for o in outs).cpu().numpy().view(np.uint64)
        assert (col % 4 == 0).all(), "column sums must be multiples of 4"
        T4 = int(col.sum()) // 4
        visited = sum(visited_sets(v, G, 4) for G in Gs)
        assert visited == T4, f"sets visited one by one ({visited}) != sets counted ({T4})"
        ref = [o.clone() for o in outs]
        if args.no_per_graph:
            return _batch_result(args, graphs, Gs, T4, visited, ms_batch, dev_ms, choice, None, None, None), graphs
        # per-graph launches, back to back on one stream
        reps = max(1, args.steps // 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for G, o in zip(Gs, outs):
                v.count(G, 4, o, stream=stream)
        stream.synchronize()
        ms_single = (time.perf_counter() - t0) * 1e3 / reps
        # per-graph, host-synchronised after every graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for G, o in zip(Gs, outs):
            v.count(G, 4, o, stream=stream)
            stream.synchronize()
        ms_sync = (time.perf_counter() - t0) * 1e3
        same = all(bool(torch.equal(a, b)) for a, b in zip(ref, outs))
    assert same, "batched and per-graph outputs differ"
    log(f"[bench] per-graph {ms_single:.1f} ms, host-synced {ms_sync:.1f} ms")
    return _batch_result(args, graphs, Gs, T4, visited, ms_batch, dev_ms, choice, ms_single, ms_sync, same), graphs


def cpu_baseline_five(graphs, budget_s):
    """The oracle (as it is) for k = 5 on the first graphs of the workload until about
    budget_s/2 of work on every host core, then on one core for about budget_s/2."""
    import oracle
    threads = oracle.default_threads()
    res = {}
    for label, th in (("all", threads), ("one", 1)):
        t0 = time.perf_counter()
        sets, done = 0, 0
        for g in graphs:
            _, tot = oracle.count(g.n, g.src, g.dst, 5, threads=th)
            sets += int(tot.sum())
            done += 1
            if time.perf_counter() - t0 > budget_s / 2:
                break
        res[label] = (sets, done, time.perf_counter() - t0)
    sets, done, secs = res["all"]
    s1, d1, t1 = res["one"]
    return {"value": sets / secs, "unit": "5-vertex sets/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle ESU + 120-relabelling class table, full k=5 count of the first {done} graphs "
                      f"({sets} sets) in {secs:.1f} s on {threads} threads",
            "one_core": {"value": s1 / t1, "graphs": d1, "sets": s1, "seconds": t1},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def bench_batch5(args, torch, gg, v):
    """k = 5 on the first 256 graphs of the batch recipe: one batched launch per step."""
    C5 = v.num_classes(5)
    graphs = gg.er_batch(256, 20, 500, 2.0, 8.0, seed=3)
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    assert all(v.count_supported(G, 5) for G in Gs)
    outs = [torch.empty((g.n, C5), dtype=torch.int64, device="cuda") for g in graphs]
    log(f"[bench] k=5 batch: {len(graphs)} graphs, {sum(g.n for g in graphs)} vertices, "
        f"outputs {8.0 * C5 * sum(g.n for g in graphs) / 2**30:.2f} GiB")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for w in range(args.warmup):
            v.count_batch(Gs, 5, outs=outs, stream=stream)
            stream.synchronize()
            log(f"[bench] warmup {w} done")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            v.count_batch(Gs, 5, outs=outs, stream=stream)
        ev1.record(stream)
        stream.synchronize()
        ms_batch = (time.perf_counter() - t0) * 1e3 / args.steps
        dev_ms = ev0.elapsed_time(ev1) / args.steps
        log(f"[bench] {args.steps} batched k=5 steps: {ms_batch:.3f} ms/step (device {dev_ms:.3f} ms)")
        col = sum(o.sum(dim=0) for o in outs).cpu().numpy().view(np.uint64)
        assert (col % 5 == 0).all(), "column sums must be multiples of 5"
        T5 = int(col.sum()) // 5
        shapes = {}
        for G in Gs:
            for key, val in v.shape_counts5(G).items():
                shapes[key] = shapes.get(key, 0) + val
        visited = sum(shapes.values())
        assert visited == T5, f"sets visited one by one ({visited}) != sets counted ({T5})"
        per_graph, same = None, None
        if not args.no_per_graph:
            ref = [o.clone() for o in outs]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for G, o in zip(Gs, outs):
                v.count(G, 5, o, stream=stream)
            stream.synchronize()
            ms_single = (time.perf_counter() - t0) * 1e3
            same = all(bool(torch.equal(a, b)) for a, b in zip(ref, outs))
            assert same, "batched and per-graph outputs differ"
            del ref
            per_graph = {"sets_per_s": T5 / (ms_single * 1e-3), "ms": ms_single}
            log(f"[bench] per-graph {ms_single:.1f} ms")
    out_bytes = 8.0 * C5 * sum(g.n for g in graphs)
    csr_bytes = sum(4.0 * (G.n + 1) + 8.0 * G.pairs + 4.0 * G.n for G in Gs)
    secs = dev_ms * 1e-3
    result = {
        "metric": "connected 5-vertex subgraphs counted/s (bit-exact), batched",
        "value": T5 / (ms_batch * 1e-3), "unit": "5-vertex sets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": WORKLOADS["batch256_k5"], "graphs": len(graphs),
                   "vertices": sum(g.n for g in graphs), "arcs": int(sum(G.arcs for G in Gs)), "sets5": T5,
                   "sets_visited": visited, "shapes_visited": shapes},
        "batched": {"sets_per_s": T5 / (ms_batch * 1e-3), "ms": ms_batch, "device_ms": dev_ms},
        "per_graph": per_graph, "batched_equals_per_graph": same,
        "roofline": roofline("batch256_k5", T5, dev_ms, "k_five (layered search) + k_five_prep + k_five_reduce",
                             out_bytes + csr_bytes, ops_per_set=MODEL_OPS_PER_SET5),
    }
    return result, graphs


def bench_graph5(args, torch, gg, v):
    """k = 5 on one graph that one workgroup's LDS does not hold: one count per step."""
    g = gg.config_graph("chunglu_5000")
    G = v.Graph(g.n, g.src, g.dst)
    out = torch.empty((g.n, v.num_classes(5)), dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for w in range(args.warmup):
            v.count(G, 5, out, stream=stream)
            stream.synchronize()
            log(f"[bench] warmup {w} done")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            v.count(G, 5, out, stream=stream)
        ev1.record(stream)
        stream.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        dev_ms = ev0.elapsed_time(ev1) / args.steps
    col = out.sum(dim=0).cpu().numpy().view(np.uint64)
    assert (col % 5 == 0).all()
    T5 = int(col.sum()) // 5
    shapes = v.shape_counts5(G)
    assert sum(shapes.values()) == T5, "sets visited one by one != sets counted"
    log(f"[bench] {args.steps} steps: {ms:.1f} ms/step, T5={T5}")
    result = {
        "metric": "connected 5-vertex subgraphs counted/s (bit-exact)", "value": T5 / (ms * 1e-3),
        "unit": "5-vertex sets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": WORKLOADS["chunglu5000_k5"], "n": g.n, "arcs": G.arcs, "pairs": G.pairs,
                   "max_degree": G.max_deg, "sets5": T5, "shapes_visited": shapes},
        "roofline": roofline("chunglu5000_k5", T5, dev_ms, "k_five_global (layered search in device memory)",
                             4.0 * (g.n + 1) + 8.0 * G.pairs + 8.0 * g.n * v.num_classes(5),
                             ops_per_set=MODEL_OPS_PER_SET5),
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline_rows(g, args.cpu_budget, k=5)
    return result


def _batch_result(args, graphs, Gs, T4, visited, ms_batch, dev_ms, choice, ms_single, ms_sync, same):
    out_bytes = 8.0 * 199 * sum(g.n for g in graphs)
    csr_bytes = sum(4.0 * (G.n + 1) + 8.0 * G.pairs for G in Gs)
    per_graph = None
    if ms_single is not None:
        per_graph = {"sets_per_s": T4 / (ms_single * 1e-3), "ms": ms_single, "host_synced_ms": ms_sync,
                     "host_synced_sets_per_s": T4 / (ms_sync * 1e-3)}
    result = {
        "metric": "connected 4-vertex subgraphs counted/s (bit-exact), batched vs per-graph; p99",
        "value": T4 / (ms_batch * 1e-3), "unit": "4-vertex sets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": WORKLOADS["batch4096"], "graphs": 4096, "vertices": sum(g.n for g in graphs),
                   "arcs": int(sum(G.arcs for G in Gs)), "sets4": T4, "sets_visited": visited},
        "batched": {"sets_per_s": T4 / (ms_batch * 1e-3), "ms": ms_batch, "device_ms": dev_ms, "tuned": choice},
        "per_graph": per_graph,
        "batched_speedup": ms_single / ms_batch if ms_single else None, "batched_equals_per_graph": same,
        "roofline": roofline("batch4096", T4, dev_ms, "k_small (whole-graph kernel) + k_batch_zero",
                             csr_bytes + out_bytes),
    }
    return result


def run_serve(v, torch, gg, pool_graphs, requests, log_hi, rates, seed=5):
    """Serving: a pool of resident graphs; requests with seeded Poisson arrivals at each rate
    (a fraction of the measured capacity); every served result equal to the alone result."""
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    pool = gg.serve_pool(pool_graphs, 2.0, log_hi, 2.0, 10.0, seed=seed)
    log(f"[bench] serve pool: {len(pool)} graphs, n <= {max(g.n for g in pool)}, "
        f"{sum(g.m for g in pool)} arcs, generated in {time.perf_counter() - t0:.1f}s")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in pool]
    picks = rng.integers(0, len(pool), size=requests)
    ks = rng.choice([3, 4], size=requests)
    # alone: every (graph, k) once, timed one at a time; capacity = 1 / mean service time
    alone, service = {}, []
    need = sorted(set(zip(picks.tolist(), ks.tolist())))
    t0 = time.perf_counter()
    for gi, k in need:
        torch.cuda.synchronize()
        t = time.perf_counter()
        o = v.count(Gs[gi], k)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t)
        alone[(gi, k)] = o
    log(f"[bench] alone pass over {len(need)} (graph, k) in {time.perf_counter() - t0:.1f}s")
    weights = np.array([sum(1 for p, k in zip(picks, ks) if (p, k) == key) for key in need], np.float64)
    mean_service = float(np.dot(weights, service) / weights.sum())
    runs = []
    for frac in rates:
        lam = frac / mean_service
        gaps = rng.exponential(1.0 / lam, size=requests)
        srv = v.Server(mem_budget_bytes=64 << 30, max_inflight=16)
        outs = [torch.empty((pool[gi].n, v.num_classes(int(k))), dtype=torch.int64, device="cuda")
                for gi, k in zip(picks, ks)]
        torch.cuda.synchronize()
        ids = []
        t_start = time.perf_counter()
        t_next = t_start
        for i in range(requests):
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                time.sleep(min(1e-4, max(0.0, t_next - time.perf_counter())))
            ids.append(srv.submit(Gs[picks[i]], int(ks[i]), outs[i]))
        for rid in ids:
            srv.wait(rid)
        wall = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        bad = sum(int(not torch.equal(outs[i], alone[(int(picks[i]), int(ks[i]))])) for i in range(requests))
        assert bad == 0, f"{bad} served results differ from the alone results"
        runs.append({"load": frac, "arrival_rate_per_s": lam, "wall_s": wall, "sets_per_s": st["sets"] / wall,
                     "req_per_s": st["req_per_s"], "p50_ms": st["p50_us"] / 1e3, "p99_ms": st["p99_us"] / 1e3,
                     "sets": st["sets"], "served_equals_alone": True,
                     "max_queue_depth": st.get("max_queue_depth"), "admitted": st.get("admitted"),
                     "deferred_by_memory": st.get("deferred_by_memory")})
        log(f"[bench] serve at {frac}x capacity: p50 {st['p50_us'] / 1e3:.2f} ms, p99 {st['p99_us'] / 1e3:.2f} ms, "
            f"{st['sets'] / wall:.3e} sets/s over {wall:.1f}s")
    # the same quantiles of the requests' alone service times (each (graph, k) weighted by its
    # number of requests): the part of the served latency that the request mix itself fixes
    order = np.argsort(service)
    cum = np.cumsum(weights[order]) / weights.sum()
    alone_q = {q: float(np.asarray(service)[order][min(int(np.searchsorted(cum, q)), len(order) - 1)]) * 1e3
               for q in (0.5, 0.99)}
    return {"workload": WORKLOADS["serve"], "pool_graphs": len(pool), "n_log10_range": [2.0, log_hi],
            "requests": requests, "mean_alone_service_ms": mean_service * 1e3,
            "alone_p50_ms": alone_q[0.5], "alone_p99_ms": alone_q[0.99], "runs": runs}


def bench_graph(args, torch, gg, v):
    """One large graph: device build + count per step."""
    t0 = time.perf_counter()
    undirected = args.workload == "chunglu_u"
    g = gg.config_graph("chunglu" if undirected else args.workload)
    log(f"[bench] generated {args.workload}: n={g.n} arcs={g.m} in {time.perf_counter() - t0:.1f}s")
    dsrc = torch.from_numpy(g.src).cuda()
    ddst = torch.from_numpy(g.dst).cuda()
    only4 = args.workload in ("rmat22", "chunglu_u")
    out3 = torch.empty((g.n if not only4 else 1, 13), dtype=torch.int64, device="cuda")
    out4 = torch.empty((g.n, 6 if undirected else 199), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    kt_steps = []

    def step(progress=False):
        G = v.Graph(g.n, dsrc, ddst, stream=stream, undirected=undirected)
        if undirected:
            v.count_undirected(G, 4, out4, stream=stream)
        elif only4:
            # one count issued as consecutive root-rank ranges (Lemma 1: independent) so that a
            # long run reports progress
            bounds = [0] + [1 << b for b in range(8, 40) if (1 << b) < g.n] + [g.n]
            for i in range(len(bounds) - 1):
                v.count_range(G, 4, out4, bounds[i], bounds[i + 1], accumulate=i > 0, stream=stream)
                if progress:
                    stream.synchronize()
                    kt_steps.append(v.kernel_times(G))
                    log(f"[bench] ranks [{bounds[i]}, {bounds[i + 1]}) done")
        else:
            v.count34(G, out3, out4, stream=stream)
        return G

    for w in range(args.warmup):
        step(progress=True)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} done")
    graphs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graphs.append(step(progress=only4))
        if not only4:
            stream.synchronize()
            kt_steps.append(v.kernel_times(graphs[-1]))
            log(f"[bench] step done: {kt_steps[-1]}")
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    G = graphs[-1]
    c4 = out4.sum(dim=0).cpu().numpy().view(np.uint64)
    assert (c4 % 4 == 0).all()
    T4 = int(c4.sum()) // 4
    if not undirected:
        assert visited_sets(v, G, 4) == T4, "k=4 sets visited one by one != sets counted"
    T3 = 0
    if not only4:
        c3 = out3.sum(dim=0).cpu().numpy().view(np.uint64)
        assert (c3 % 3 == 0).all()
        T3 = int(c3.sum()) // 3
        assert visited_sets(v, G, 3) == T3, "k=3 sets visited one by one != sets counted"
    # kernel times (HIP events the library records on the stream): one record per timed step,
    # or one per root range of each step for the ranged count
    timed = kt_steps[-(len(kt_steps) * args.steps // (args.steps + (args.warmup if only4 else 0))):]
    light = sum(max(0.0, k[0]) for k in timed) / args.steps
    hub = sum(max(0.0, k[1]) for k in timed) / args.steps
    khub = sum(max(0.0, k[2]) for k in timed) / args.steps
    log(f"[bench] {args.steps} steps: {ms_step:.1f} ms/step, T4={T4} T3={T3}")
    sc = v.shape_counts(G)
    csr_bytes = 4.0 * (g.n + 1) + 8.0 * G.pairs
    result = {
        "metric": "connected 4-vertex subgraphs counted/s (bit-exact)", "value": T4 / (ms_step * 1e-3),
        "unit": "4-vertex sets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n": g.n, "arcs": G.arcs, "pairs": G.pairs,
                   "max_degree": G.max_deg, "sets3": T3, "sets4": T4, "shapes_visited": sc},
        "sets3_per_s": T3 / (ms_step * 1e-3), "light_ms": light, "hub_path_ms": hub, "k_hub_ms": khub,
    }
    if hub:
        result["roofline"] = roofline(args.workload, T4 + T3, hub + (light or 0.0),
                                      "hub path (k_hub + k_long_slots) + per-root kernel",
                                      csr_bytes + 8.0 * g.n * (13 + 199))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline ...")
        gb = g if not undirected else gg.Graph(g.n, np.concatenate([g.src, g.dst]),
                                               np.concatenate([g.dst, g.src]), "chunglu_u")
        result["cpu_baseline"] = cpu_baseline_rows(gb, args.cpu_budget)
    return result


def calibrate_copy(torch):
    """Reference readings for the HBM byte counters: a plain 1 GiB device-to-device copy."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log("[bench] calibration copy of 1 GiB done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch4096", choices=sorted(WORKLOADS))
    ap.add_argument("--serve-graphs", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-log-hi", type=float, default=None,
                    help="pool n up to 10^this (default: 4.5 in the default run, 6 for --workload serve)")
    ap.add_argument("--no-serve", action="store_true", help="default run without the serving leg")
    ap.add_argument("--no-per-graph", action="store_true",
                    help="default run without the per-graph comparison (for profiler runs)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--only-calibrate-copy", action="store_true",
                    help="run the 1 GiB reference copy alone (for the HBM byte counters) and exit")
    ap.add_argument("--tune-cache", default=None,
                    help="file the autotuner appends its choice to (read back through VDMC_TUNE_CACHE)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the per-vertex motif count here is a single-GPU build "
              "(multi-GPU sharding is described in the design notes, not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as gg
    import paper_2201_11655_amd as v

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.only_calibrate_copy:
        calibrate_copy(torch)
        return
    v.load()
    if args.workload == "batch4096":
        result, graphs = bench_batch(args, torch, gg, v)
        if not args.no_serve:
            log_hi = 4.5 if args.serve_log_hi is None else args.serve_log_hi
            result["serve"] = run_serve(v, torch, gg, args.serve_graphs, args.serve_requests, log_hi, (0.5, 0.8))
        if not args.no_cpu_baseline:
            log("[bench] cpu baseline ...")
            result["cpu_baseline"] = cpu_baseline_batch(graphs, args.cpu_budget)
    elif args.workload == "batch256_k5":
        result, graphs = bench_batch5(args, torch, gg, v)
        if not args.no_cpu_baseline:
            log("[bench] cpu baseline ...")
            result["cpu_baseline"] = cpu_baseline_five(graphs, args.cpu_budget)
    elif args.workload == "chunglu5000_k5":
        result = bench_graph5(args, torch, gg, v)
    elif args.workload == "serve":
        log_hi = 6.0 if args.serve_log_hi is None else args.serve_log_hi
        s = run_serve(v, torch, gg, args.serve_graphs, args.serve_requests, log_hi, (0.5, 0.8))
        r8 = s["runs"][-1]
        result = {"metric": "served k-vertex sets counted/s (bit-exact); p50/p99 latency",
                  "value": r8["sets_per_s"], "unit": "sets/s", "n_gpus": 1, "steps": args.serve_requests,
                  "warmup": 0, "ms_per_step": r8["wall_s"] * 1e3 / args.serve_requests, "higher_is_better": True,
                  "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
                  "config": {"workload": WORKLOADS["serve"]}, "serve": s}
    else:
        result = bench_graph(args, torch, gg, v)
    if args.calibrate_copy:
        calibrate_copy(torch)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
