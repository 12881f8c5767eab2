"""GPU parity for 5-vertex motifs (the Sec. 11 extension): the HIP path through the C ABI
against the CPU oracle, every uint64 entry equal.

Covers the class table (2^20 codes, 9364 classes), single-graph counts (parts of one
graph sharing its items, each with its own LDS counters and output block), batched counts
with many small graphs (most of them one part each) and with few larger ones (many parts
each), graphs too large for LDS (counted in device memory, device-scope credits), mixed
batches, the count limits of the per-lane credit caches, the visited-set counters per BFS
layer shape and the degenerate cases (n < 5, no arcs, self-loops, isolated vertices).
"""
import math
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

C5 = 9364


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
    sys.stdout.flush()


def _check(v, n, src, dst, label):
    _say(f"k=5 case {label} n={n} m={len(src)}")
    G = v.Graph(n, src, dst)
    got = _np(v.count(G, 5))
    want, tot = oracle.count(n, src, dst, 5)
    assert got.shape == want.shape == (n, C5)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{label}: {bad.shape[0]} cells differ, first {bad[:5].tolist()}"
    sc = v.shape_counts5(G)
    assert sum(sc.values()) == int(tot.sum()), (label, sc, int(tot.sum()))
    return G, sc


def test_class_table_k5(v):
    canon, cls, codes = oracle.class_table(5)
    assert v.num_classes(5) == C5
    assert (v.class_codes(5) == codes.astype(np.uint32)).all()
    t = v.class_table(5)
    want = np.where(cls >= 0, cls, 0xFFFF).astype(np.uint16)
    assert (t == want).all()
    # the k = 3, 4 tables in the wide form agree with the narrow ones
    for k in (3, 4):
        lib = v.load()
        import ctypes
        wide = np.zeros(1 << (k * (k - 1)), np.uint16)
        assert lib.vdmc_class_table_u16(k, wide.ctypes.data_as(ctypes.c_void_p)) == 0
        narrow = v.class_table(k).astype(np.uint16)
        assert (wide == np.where(narrow == 0xFF, 0xFFFF, narrow)).all()


@pytest.mark.parametrize("case", [
    ("er", 37, 0.2, 1), ("er", 120, 0.05, 2), ("er", 300, 0.012, 3), ("er", 64, 0.5, 4),
    ("er", 512, 0.006, 5), ("er", 200, 0.03, 6),
])
def test_parity_random(v, case):
    _, n, p, seed = case
    g = gg.er_directed(n, p, (90, seed))
    _check(v, n, g.src, g.dst, f"er({n},{p})")


def test_parity_skewed_degrees(v):
    """A Chung-Lu graph with hubs (roots with many higher neighbours, long items)."""
    g = gg.chung_lu(400, 1600, 2.1, 60.0, 0.2, 120, (91, 1))
    _, sc = _check(v, g.n, g.src, g.dst, "chunglu(400)")
    assert all(x > 0 for x in sc.values())


@pytest.mark.parametrize("name", ["complete", "tournament", "outstar", "instar", "cycle"])
def test_closed_forms(v, name):
    """K_n, the transitive tournament and stars: every 5-set is one motif; a vertex lies in
    C(n-1, 4) of them (a star's leaves in C(n-2, 3)).  Directed n-cycle: n windows."""
    n = 13
    g = gg.special_graph(name, n)
    G, sc = _check(v, n, g.src, g.dst, name)
    got = _np(v.count(G, 5))
    if name in ("complete", "tournament"):
        assert (got.sum(axis=1) == math.comb(n - 1, 4)).all() and sc["(4)"] == math.comb(n, 5)
    elif name in ("outstar", "instar"):
        assert got[0].sum() == math.comb(n - 1, 4) and (got[1:].sum(axis=1) == math.comb(n - 2, 3)).all()
    else:
        assert (got.sum(axis=1) == 5).all() and sum(sc.values()) == n


def test_star_past_cache_limits(v):
    """An out-star on 1030 vertices (device-memory path): one context holds 1026 last
    members of one signature and one depth-2 loop over 5e5 sets of one class, past the
    count limits of both per-lane credit caches (1023 and 2^18), so their overflow paths
    run.  Closed form: the hub lies in C(n-1, 4) sets, a leaf in C(n-2, 3), all of the
    out-star class (read from the oracle's count of a 6-vertex out-star)."""
    n = 1030
    g = gg.special_graph("outstar", n)
    small = gg.special_graph("outstar", 6)
    want6, _ = oracle.count(6, small.src, small.dst, 5)
    cls = int(np.flatnonzero(want6[0])[0])
    _say(f"k=5 out-star n={n}: {math.comb(n - 1, 4)} sets")
    G = v.Graph(n, g.src, g.dst)
    got = _np(v.count(G, 5))
    exp = np.zeros((n, C5), np.uint64)
    exp[0, cls] = math.comb(n - 1, 4)
    exp[1:, cls] = math.comb(n - 2, 3)
    assert (got == exp).all()
    assert sum(v.shape_counts5(G).values()) == math.comb(n - 1, 4)


def test_degenerate(v):
    for n, src, dst, label in [
        (4, [0, 1, 2], [1, 2, 3], "n<5"),
        (9, [], [], "no arcs"),
        (9, list(range(9)), list(range(9)), "self-loops only"),
        (12, [0, 1, 2, 3], [1, 2, 3, 4], "path plus isolated vertices"),
    ]:
        s = np.array(src, np.int32)
        d = np.array(dst, np.int32)
        _check(v, n, s, d, label)


def test_batch_owned_mode(v):
    """More graphs than compute units, most of them small: parts are few per graph (one for
    graphs with fewer than 64 pairs)."""
    import torch
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    gs = gg.er_batch(ncu + 20, 5, 120, 1.0, 5.0, seed=92)
    gs[3] = gg.er_directed(3, 0.9, (92, 3))        # n < 5
    gs[7] = gg.Graph(6, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty")
    _say(f"k=5 batch owned: {len(gs)} graphs, {sum(g.n for g in gs)} vertices")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in gs]
    for rep in range(2):   # a second call reuses the cached launch and re-zeroes everything
        outs = v.count_batch(Gs, 5)
        for i, (g, G, o) in enumerate(zip(gs, Gs, outs)):
            want, tot = oracle.count(g.n, g.src, g.dst, 5, threads=4)
            assert (_np(o) == want).all(), (rep, i)
            assert sum(v.shape_counts5(G).values()) == int(tot.sum()), (rep, i)


def test_batch_shared_mode(v):
    """Fewer graphs than compute units: each graph cut into many parts over the grid."""
    gs = gg.er_batch(9, 30, 400, 2.0, 6.0, seed=93)
    _say(f"k=5 batch shared: {len(gs)} graphs")
    Gs = [v.Graph(g.n, g.src, g.dst) for g in gs]
    outs = v.count_batch(Gs, 5)
    for i, (g, o) in enumerate(zip(gs, outs)):
        want, _ = oracle.count(g.n, g.src, g.dst, 5)
        assert (_np(o) == want).all(), i


@pytest.mark.parametrize("case", [("er", 1200, 0.004, 1), ("er", 3000, 0.0015, 2),
                                  ("chunglu", 800, 3200, 40.0), ("chunglu", 1500, 4500, 30.0)])
def test_parity_device_memory_path(v, case):
    """Graphs that one workgroup's LDS does not hold (n > 512): the search runs over the
    graph in device memory (edge-hash pair tests, one shared item cursor, device-scope
    credits)."""
    if case[0] == "er":
        _, n, p, seed = case
        g = gg.er_directed(n, p, (95, seed))
    else:
        _, n, m, wcap = case
        g = gg.chung_lu(n, m, 2.1, wcap, 0.2, int(2 * wcap), (96, n))
    G, sc = _check(v, g.n, g.src, g.dst, f"{case[0]}({g.n}) in device memory")
    assert G.n > 512


def test_batch_mixed_lds_and_device_memory(v):
    """A batch whose graphs are partly too large for LDS: the LDS ones in the batched
    launch, the others counted in device memory after it; all equal to the oracle."""
    gs = gg.er_batch(12, 30, 300, 2.0, 5.0, seed=97)
    gs[2] = gg.er_directed(900, 0.005, (97, 2))
    gs[7] = gg.er_directed(700, 0.006, (97, 7))
    Gs = [v.Graph(g.n, g.src, g.dst) for g in gs]
    outs = v.count_batch(Gs, 5)
    for i, (g, G, o) in enumerate(zip(gs, Gs, outs)):
        want, tot = oracle.count(g.n, g.src, g.dst, 5)
        assert (_np(o) == want).all(), i
        assert sum(v.shape_counts5(G).values()) == int(tot.sum()), i


def test_limits_and_errors(v):
    import ctypes
    lib = v.load()
    g = gg.er_directed(40, 0.1, (94, 1))
    G = v.Graph(g.n, g.src, g.dst)
    assert v.count_supported(G, 5) and v.count_supported(G, 4)
    assert lib.vdmc_count_supported(G.handle, 6) == -1
    with pytest.raises(v.VdmcError) as e:
        v.count(G, 6)
    assert e.value.name == "INVALID_ARG"
    rc = lib.vdmc_count(G.handle, 5, None, None)
    assert rc == 1   # NULL output
    empty = v.Graph(600, np.zeros(0, np.int32), np.zeros(0, np.int32))   # device-memory path, no arcs
    o = v.count(empty, 5)
    assert int(_np(o).sum()) == 0 and sum(v.shape_counts5(empty).values()) == 0
