"""GPU tests of the batched launch (many graphs, one persistent captured launch, tuner)
and of the serving loop (continuous batching, memory admission).  Every count is
compared bit-exactly with the oracle or with the single-graph path."""
import os
import sys
import tempfile

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def v():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_11655_amd as v
    v.load()
    return v


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def small_batch():
    # same recipe as the 4096-graph batch workload, fewer graphs
    return gg.er_batch(48, 20, 500, 2.0, 8.0, seed=3)


@pytest.mark.parametrize("k", [3, 4])
def test_batch_equals_oracle(v, small_batch, k):
    import torch
    _say(f"batch k={k} graphs={len(small_batch)}")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in small_batch]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = v.count_batch(Gs, k, stream=stream)
        stream.synchronize()
        for rep in range(3):   # replays of the captured launch, with eager work in between
            for o in outs:
                o.fill_(-1)
            torch.cuda.synchronize()
            v.count_batch(Gs, k, outs=outs, stream=stream)
            stream.synchronize()
            for g, o in zip(small_batch, outs):
                want, _ = oracle.count(g.n, g.src, g.dst, k)
                assert (_np(o) == want).all(), f"replay {rep} graph n={g.n}"


@pytest.mark.parametrize("k", [3, 4])
def test_batch_small_graph_edge_cases(v, k):
    # graphs taken whole by one workgroup: no arcs, one vertex, the largest size taken
    # that way (1024), a dense graph whose roots exceed the hub threshold, and one just
    # above the size limit (counted root by root)
    import torch
    graphs = [gg.er_directed(1, 0.0, (61, 0)), gg.er_directed(7, 0.0, (61, 1)),
              gg.er_directed(1024, 6.0 / 1023, (61, 2)), gg.er_directed(200, 0.15, (61, 3)),
              gg.er_directed(1025, 5.0 / 1024, (61, 4)), gg.er_directed(3, 0.9, (61, 5))]
    _say(f"batch edge cases k={k} n={[g.n for g in graphs]}")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = v.count_batch(Gs, k, stream=stream)
        stream.synchronize()
    for g, o in zip(graphs, outs):
        want, _ = oracle.count(g.n, g.src, g.dst, k)
        assert (_np(o) == want).all(), f"graph n={g.n} arcs={g.m}"


@pytest.mark.parametrize("k", [3, 4])
def test_batch_special_and_dense_graphs(v, k):
    """Whole-graph counts of graphs whose sets fall almost all outside the LDS counter
    slots (complete bidirected graph, transitive tournament, dense G(n,p) with many
    reciprocal pairs) or all inside them (cycle, stars, path), in one batch."""
    import torch
    graphs = [gg.special_graph(kind, 13) for kind in ("complete", "tournament", "cycle", "outstar", "instar", "path")]
    graphs += [gg.er_directed(64, 0.5, (62, 0)), gg.er_directed(40, 0.3, (62, 1)), gg.er_directed(90, 0.08, (62, 2))]
    _say(f"batch special/dense k={k} n={[g.n for g in graphs]}")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = v.count_batch(Gs, k, stream=stream)
        stream.synchronize()
    for g, o in zip(graphs, outs):
        want, _ = oracle.count(g.n, g.src, g.dst, k)
        assert (_np(o) == want).all(), f"graph {g.name}"


def test_batch_with_hub_graph_and_single_path(v, small_batch):
    import torch
    graphs = small_batch[:8] + [gg.config_graph("chunglu_2000")] + small_batch[8:12]
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = v.count_batch(Gs, 4, stream=stream)
        stream.synchronize()
    for G, o in zip(Gs, outs):
        single = _np(v.count(G, 4))
        assert (_np(o) == single).all()


def test_tune_and_cache(v, small_batch):
    import torch
    Gs = [v.Graph(g.n, g.src, g.dst) for g in small_batch[:16]]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        assert not v.tuned_choice(Gs, 4)["tuned"]
        v.tune(Gs, 4, path)
        fields = open(path).read().split()
        # k, graphs, vertices, pairs, small-kernel variant, root variant, workgroups/CU, tile, ms
        assert len(fields) == 9 and fields[:4] == ["4", "16", str(sum(g.n for g in Gs)), str(sum(g.pairs for g in Gs))]
        c = v.tuned_choice(Gs, 4)
        assert c["tuned"] and c["small_threads"] in (256, 512, 1024)
        assert not v.tuned_choice(Gs[:15], 4)["tuned"]   # another batch shape keeps the defaults
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = v.count_batch(Gs, 4, stream=stream)
        stream.synchronize()
    for g, o in zip(small_batch[:16], outs):
        want, _ = oracle.count(g.n, g.src, g.dst, 4)
        assert (_np(o) == want).all()


def test_batch_errors(v, small_batch):
    Gs = [v.Graph(g.n, g.src, g.dst) for g in small_batch[:2]]
    with pytest.raises(v.VdmcError) as e:
        v.count_batch(Gs, 6)
    assert e.value.name == "INVALID_ARG"
    assert v.count_batch([], 4) == []


# --------------------------------------------------------------------------- serving

def _pool():
    pool = [gg.er_directed(int(n), mu / (n - 1), (51, i)) for i, (n, mu) in
            enumerate([(120, 3), (400, 5), (60, 8), (900, 4), (250, 2.5), (30, 6)])]
    pool.append(gg.config_graph("chunglu_2000"))
    pool.append(gg.config_graph("er1000"))
    return pool


def test_serve_alone_equals_mix(v):
    import torch
    pool = _pool()
    Gs = [v.Graph(g.n, g.src, g.dst) for g in pool]
    rng = np.random.default_rng(7)
    reqs = [(int(rng.integers(len(pool))), int(rng.choice([3, 4]))) for _ in range(40)]
    # alone: each request by itself through vdmc_count
    alone = {}
    for gi, k in set(reqs):
        alone[(gi, k)] = _np(v.count(Gs[gi], k)).copy()
    srv = v.Server(mem_budget_bytes=8 << 30, max_inflight=6)
    outs, ids = [], []
    for gi, k in reqs:
        o = torch.empty((pool[gi].n, v.num_classes(k)), dtype=torch.int64, device="cuda")
        outs.append(o)
        ids.append(srv.submit(Gs[gi], k, o))
    for rid in ids:
        srv.wait(rid)
        assert srv.poll(rid)
    torch.cuda.synchronize()
    for (gi, k), o in zip(reqs, outs):
        assert (_np(o) == alone[(gi, k)]).all(), f"graph {gi} k={k} differs in the mix"
    st = srv.stats()
    assert st["p50_us"] > 0 and st["p99_us"] >= st["p50_us"] and st["req_per_s"] > 0
    expect_sets = sum(int(alone[(gi, k)].sum()) // k for gi, k in reqs)
    assert st["sets"] == expect_sets
    srv.close()


def _hub_graphs(count):
    # Chung-Lu graphs of the benchmark recipe at n = 2,000: every one has hub roots, so a
    # request on it needs the hub path's scratch
    return [gg.chung_lu(2000, 16800, 2.1, 45.0, 0.2, 90, (77, i)) for i in range(count)]


def test_serve_admission_and_errors(v):
    import torch
    hubs = _hub_graphs(1)[0]
    G = v.Graph(hubs.n, hubs.src, hubs.dst)
    out = torch.empty((hubs.n, 199), dtype=torch.int64, device="cuda")
    tiny = v.Server(mem_budget_bytes=1 << 16, max_inflight=2)   # smaller than the hub scratch
    rid = tiny.submit(G, 4, out)             # the graph's bins are built at its first admission
    with pytest.raises(v.VdmcError) as e:
        tiny.wait(rid)
    assert e.value.name == "REJECTED"
    with pytest.raises(v.VdmcError) as e:    # bins known now: refused at submit
        tiny.submit(G, 4, out)
    assert e.value.name == "REJECTED"
    with pytest.raises(v.VdmcError) as e:
        tiny.poll(12345)
    assert e.value.name == "NOT_FOUND"
    with pytest.raises(v.VdmcError) as e:
        tiny.submit(G, 5, out)
    assert e.value.name == "UNSUPPORTED"
    c = tiny.stats()
    assert c["rejected"] == 1 and c["completed"] == 0
    tiny.close()


def test_serve_budget_holds_requests_back(v):
    """The memory budget, not max_inflight, limits what runs: the budget fits the hub
    scratch of one request at a time, so later requests wait for memory; every result
    equals the alone count and the server never holds more than the budget."""
    import torch
    graphs = _hub_graphs(4)
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    alone = [_np(v.count(G, 4)).copy() for G in Gs]
    # the alone counts keep each graph's scratch: served requests start from new graphs;
    # one probe server per graph measures the scratch a request on it needs
    needs = []
    for g in graphs:
        G = v.Graph(g.n, g.src, g.dst)
        probe = v.Server(mem_budget_bytes=1 << 40, max_inflight=1)
        o = torch.empty((g.n, 199), dtype=torch.int64, device="cuda")
        probe.wait(probe.submit(G, 4, o))
        needs.append(probe.stats()["max_bytes_in_flight"])
        probe.close()
    assert min(needs) > 0 and max(needs) < 2 * min(needs)
    budget = (max(needs) + 2 * min(needs)) // 2   # fits any one request, never two
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    srv = v.Server(mem_budget_bytes=budget, max_inflight=8)
    outs = [torch.empty((g.n, 199), dtype=torch.int64, device="cuda") for g in graphs]
    ids = [srv.submit(G, 4, o) for G, o in zip(Gs, outs)]
    for rid in ids:
        srv.wait(rid)
    st = srv.stats()
    srv.close()
    for o, a in zip(outs, alone):
        assert (_np(o) == a).all()
    assert st["completed"] == 4 and st["deferred_by_memory"] > 0
    assert st["max_bytes_in_flight"] <= budget


def test_concurrent_counts_on_one_graph(v):
    """One graph counted on two streams at once (and inside a batch on a third): every
    call's work is ordered after the previous call's on the graph, so each output equals
    the oracle."""
    import torch
    g = gg.config_graph("chunglu_2000")
    want3, _ = oracle.count(g.n, g.src, g.dst, 3)
    want4, _ = oracle.count(g.n, g.src, g.dst, 4)
    G = v.Graph(g.n, g.src, g.dst)
    small = gg.er_directed(300, 0.02, (5, 5))
    Gs = v.Graph(small.n, small.src, small.dst)
    want_s, _ = oracle.count(small.n, small.src, small.dst, 4)
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        a4 = torch.full((g.n, 199), -1, dtype=torch.int64, device="cuda")
        b4 = torch.full((g.n, 199), -1, dtype=torch.int64, device="cuda")
        b3 = torch.full((g.n, 13), -1, dtype=torch.int64, device="cuda")
        c4 = torch.full((g.n, 199), -1, dtype=torch.int64, device="cuda")
        cs = torch.full((small.n, 199), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        v.count(G, 4, a4, stream=s1)
        v.count34(G, b3, b4, stream=s2)
        v.count_batch([Gs, G], 4, outs=[cs, c4], stream=s3)
        torch.cuda.synchronize()
        assert (_np(a4) == want4).all(), f"rep {rep}: stream 1"
        assert (_np(b4) == want4).all() and (_np(b3) == want3).all(), f"rep {rep}: stream 2"
        assert (_np(c4) == want4).all() and (_np(cs) == want_s).all(), f"rep {rep}: batch"


def test_serve_destroy_with_work_in_flight(v):
    import torch
    pool = _pool()
    Gs = [v.Graph(g.n, g.src, g.dst) for g in pool]
    srv = v.Server(mem_budget_bytes=8 << 30, max_inflight=2)
    outs = [torch.empty((g.n, 199), dtype=torch.int64, device="cuda") for g in pool]
    for G, o in zip(Gs, outs):
        srv.submit(G, 4, o)
    srv.close()          # waits for running requests, cancels queued ones
    torch.cuda.synchronize()
