"""Parity at full workload sizes, in the launch configuration the benchmark times.

The oracle cannot enumerate 1e12 sets, so these tests compare 64 rows per workload (the
16 vertices of largest degree, whose rows the hub path writes, and 48 seeded random
non-isolated vertices) with rows the oracle computed one vertex at a time
(tests/golden/fullsize_<name>.txt, written by tests/golden/make_fullsize_rows.py, keyed
by the SHA-256 of the generated input), and check properties that hold at any size:
every column sum is a multiple of k and equals k times the number of sets the kernels
visited one by one, isolated vertices have zero rows.
"""
import os
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _golden(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.txt")
    sha, rows, want = None, None, {}
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "sha256":
                sha = parts[1]
            elif parts[0] == "rows":
                rows = [int(x) for x in parts[1:]]
            else:
                vtx, k, c, cnt = (int(x) for x in parts)
                want.setdefault(k, {}).setdefault(vtx, {})[c] = cnt
    return sha, rows, want


def _check_full(v, name, ks):
    import torch
    g = gg.config_graph(name)
    sha, rows, want = _golden(name)
    assert gg.digest(g) == sha, f"{name}: the stored rows were computed on another input"
    _say(f"full-size case {name}: n={g.n} arcs={g.m}, {len(rows)} stored oracle rows")
    G = v.Graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda())
    if ks == (3, 4):
        o3, o4 = v.count34(G)
        outs = {3: o3, 4: o4}
    else:
        outs = {4: v.count(G, 4)}
    torch.cuda.synchronize()
    sc = v.shape_counts(G)
    idx = torch.from_numpy(np.array(rows, np.int64)).cuda()
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    iso = np.flatnonzero(deg == 0)[:8]
    for k, o in outs.items():
        C = v.num_classes(k)
        col = o.sum(dim=0).cpu().numpy().view(np.uint64)
        assert (col % k == 0).all()
        T = int(col.sum()) // k
        visited = sc["(1,1)"] + sc["(1,2)"] if k == 3 else \
            sc["(3,0,0)"] + sc["(2,1,0)"] + sc["(1,2,0)"] + sc["(1,1,1)"]
        assert visited == T, f"{name} k={k}: visited {visited} != counted {T}"
        got = o[idx].cpu().numpy().view(np.uint64)
        exp = np.zeros((len(rows), C), np.uint64)
        for i, r in enumerate(rows):
            for c, cnt in want[k].get(r, {}).items():
                exp[i, c] = cnt
        bad = np.argwhere(got != exp)
        assert bad.size == 0, f"{name} k={k}: {bad.shape[0]} cells differ, first rows {[rows[b[0]] for b in bad[:5]]}"
        if iso.size:
            assert (o[torch.from_numpy(iso.astype(np.int64)).cuda()].cpu().numpy() == 0).all()
        _say(f"  k={k}: T={T}, {len(rows)} rows equal the oracle's")


def test_chunglu_full_size(v):
    _check_full(v, "chunglu", (3, 4))


def test_rmat22_full_size(v):
    if not os.path.exists(os.path.join(GOLDEN, "fullsize_rmat22.txt")):
        pytest.skip("stored oracle rows of the R-MAT workload not generated")
    _check_full(v, "rmat22", (4,))


def test_batch4096_full_size(v):
    """All 4096 graphs in one batched launch; a seeded sample of 256 graphs checked against
    the oracle entirely, and every 97th graph against its own single-graph count."""
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


def test_batch256_k5_full_size(v):
    """The 5-vertex workload at full size: the first 256 graphs of the batch recipe in one
    batched launch (graphs cut into parts); the 32 graphs with the most work and 32
    seeded random others checked against the oracle entirely, every graph's visited
    counters against its column sums, and every 17th graph against its single-graph count
    (the shared mode)."""
    import torch
    graphs = gg.er_batch(256, 20, 500, 2.0, 8.0, seed=3)
    _say(f"batch256_k5: {sum(g.n for g in graphs)} vertices")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in graphs]
    outs = v.count_batch(Gs, 5)
    torch.cuda.synchronize()
    for i, (G, o) in enumerate(zip(Gs, outs)):
        col = o.sum(dim=0).cpu().numpy().view(np.uint64)
        assert (col % 5 == 0).all() and int(col.sum()) // 5 == sum(v.shape_counts5(G).values()), i
    work = np.array([G.pairs * float(G.max_deg) ** 3 for G in Gs])
    heavy = np.argsort(-work)[:32]
    rest = np.setdiff1d(np.arange(len(graphs)), heavy)
    pick = np.concatenate([heavy, np.random.default_rng(35).choice(rest, size=32, replace=False)])
    for i in pick:
        g = graphs[i]
        want, _ = oracle.count(g.n, g.src, g.dst, 5)
        assert (outs[i].cpu().numpy().view(np.uint64) == want).all(), f"graph {i}"
    _say(f"  {len(pick)} graphs equal the oracle's")
    for i in range(0, len(graphs), 17):
        assert torch.equal(v.count(Gs[i], 5), outs[i]), i
