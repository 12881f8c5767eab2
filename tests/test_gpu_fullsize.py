"""Parity at full workload sizes, in the launch configuration the benchmark times.

The oracle cannot enumerate 1e12 sets, so these tests compare seeded samples of
output rows that the oracle computes one vertex at a time (its per-vertex mode), and
check properties that hold at any size: every column sum is a multiple of k, the
per-shape set counts add up to the column sums, isolated vertices have zero rows.
"""
import sys

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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sample_rows(g, count, max_deg, seed):
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    rng = np.random.default_rng(seed)
    cand = np.flatnonzero((deg > 0) & (deg <= max_deg))
    iso = np.flatnonzero(deg == 0)
    rows = list(rng.choice(cand, size=count, replace=False))
    if iso.size:
        rows.append(int(iso[0]))
    return np.array(rows, np.int32)


def _check_full(v, name, ks, rows_per_k, seed):
    import torch
    g = gg.config_graph(name)
    _say(f"full-size case {name}: n={g.n} arcs={g.m}")
    dsrc = torch.from_numpy(g.src).cuda()
    ddst = torch.from_numpy(g.dst).cuda()
    G = v.Graph(g.n, dsrc, ddst)
    if ks == (3, 4):
        o3, o4 = v.count34(G)
        outs = {3: o3, 4: o4}
    else:
        outs = {4: v.count(G, 4)}
    torch.cuda.synchronize()
    sc = v.shape_counts(G)
    rows = _sample_rows(g, rows_per_k, 4, seed)
    for k, o in outs.items():
        col = o.sum(dim=0).cpu().numpy().view(np.uint64)
        assert (col % k == 0).all()
        T = int(col.sum()) // k
        if k == 3:
            assert sc["(1,1)"] + sc["(1,2)"] == T
        else:
            assert sc["(3,0,0)"] + sc["(2,1,0)"] + sc["(1,2,0)"] + sc["(1,1,1)"] == T
        got = o[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy().view(np.uint64)
        _say(f"  k={k}: T={T}, oracle rows {rows.tolist()}")
        want = oracle.count_rows(g.n, g.src, g.dst, k, rows)
        assert (got == want).all(), f"{name} k={k}: sampled rows differ"


def test_chunglu_full_size(v):
    _check_full(v, "chunglu", (3, 4), 8, 21)


def test_rmat22_full_size(v):
    _check_full(v, "rmat22", (4,), 6, 22)


def test_batch4096_full_size(v):
    """All 4096 graphs in one batched launch; a seeded sample of 256 graphs checked against
    the oracle entirely, and every graph against its own single-graph count."""
    import torch
    graphs = gg.er_batch(4096, 20, 500, 2.0, 8.0, seed=3)
    _say(f"batch4096: {sum(g.n for g in graphs)} vertices")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = v.count_batch(Gs, 4, stream=stream)
        stream.synchronize()
    pick = np.random.default_rng(33).choice(len(graphs), size=256, replace=False)
    for i in pick:
        g = graphs[i]
        want, _ = oracle.count(g.n, g.src, g.dst, 4, threads=4)
        assert (outs[i].cpu().numpy().view(np.uint64) == want).all(), f"graph {i}"
    for i in range(0, len(graphs), 97):
        single = v.count(Gs[i], 4)
        assert torch.equal(single, outs[i])
