"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

All counts are integers, so the bar is bit-exact equality of every uint64 entry.
"""
import os
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


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check_graph(v, n, src, dst, ks=(3, 4), threads=None, label=""):
    _say(f"case {label} n={n} m={len(src)}")
    G = v.Graph(n, src, dst)
    for k in ks:
        got = _np(v.count(G, k))
        want, tot = oracle.count(n, src, dst, k, threads=threads)
        assert got.shape == want.shape
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{label} k={k}: {bad.shape[0]} cells differ, first {bad[:5].tolist()}"
        sc = v.shape_counts(G)
        if k == 3:
            assert sc["(1,1)"] + sc["(1,2)"] == int(tot.sum())
        else:
            assert sc["(3,0,0)"] + sc["(2,1,0)"] + sc["(1,2,0)"] + sc["(1,1,1)"] == int(tot.sum())
    return G


# --------------------------------------------------------------------------- class table

@pytest.mark.parametrize("k", [3, 4])
def test_class_table_equals_oracle(v, k):
    canon, cls, codes = oracle.class_table(k)
    t = v.class_table(k)
    want = np.where(cls >= 0, cls, 255).astype(np.uint8)
    assert (t == want).all()
    assert (v.class_codes(k) == codes).all()


# --------------------------------------------------------------------------- graph build

def _expected_rank_csr(n, src, dst):
    off, nbr, dr = oracle.simple_graph(n, src, dst)
    deg = np.diff(off)
    perm = np.lexsort((np.arange(n), -deg))          # degree descending, id ascending
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    rows = []
    for r in range(n):
        v0 = perm[r]
        ent = sorted((int(inv[nbr[e]]) << 2) | int(dr[e]) for e in range(off[v0], off[v0 + 1]))
        rows.append(ent)
    roff = np.zeros(n + 1, np.uint32)
    roff[1:] = np.cumsum([len(x) for x in rows])
    radj = np.array([e for x in rows for e in x], np.uint32)
    return roff, radj, perm.astype(np.int32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_graph_build_matches_definition(v, seed):
    g = gg.er_directed(300, 0.02, (5, seed))
    src = np.concatenate([g.src, g.src[:50], np.array([3, 7], np.int32)])     # duplicates
    dst = np.concatenate([g.dst, g.dst[:50], np.array([3, 7], np.int32)])     # + self-loops
    G = v.Graph(g.n, src, dst)
    off, adj, perm = G.export()
    roff, radj, rperm = _expected_rank_csr(g.n, src, dst)
    assert (off == roff).all() and (adj == radj).all() and (perm == rperm).all()
    assert G.arcs == len(set(zip(g.src.tolist(), g.dst.tolist())))
    assert G.pairs == len(radj) // 2


def test_graph_build_device_input(v):
    import torch
    g = gg.er_directed(500, 0.01, 17)
    Gh = v.Graph(g.n, g.src, g.dst)
    Gd = v.Graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda())
    for a, b in zip(Gh.export(), Gd.export()):
        assert (a == b).all()


def test_csr_example_sec42(v):
    """The example graph of Sec. 4.2 in the library's CSR (ids = ranks here after the
    degree order is undone through perm)."""
    src = np.array([0, 0, 0, 2, 3, 3], np.int32)
    dst = np.array([1, 2, 3, 0, 1, 2], np.int32)
    G = v.Graph(4, src, dst)
    off, adj, perm = G.export()
    und = {}
    for r in range(4):
        und[int(perm[r])] = sorted(int(perm[e >> 2]) for e in adj[off[r]:off[r + 1]])
    assert [und[i] for i in range(4)] == [[1, 2, 3], [0, 3], [0, 3], [0, 1, 2]]


# --------------------------------------------------------------------------- counts

@pytest.mark.parametrize("seed", range(16))
def test_tiny_random_graphs(v, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 14))
    p = float(rng.uniform(0.05, 0.8))
    g = gg.er_directed(n, p, (21, seed))
    _check_graph(v, n, g.src, g.dst, label=f"tiny{seed}")


@pytest.mark.parametrize("kind", ["complete", "tournament", "cycle", "outstar", "instar", "path"])
def test_special_graphs(v, kind):
    n = 12
    g = gg.special_graph(kind, n)
    _check_graph(v, n, g.src, g.dst, label=kind)


def test_dense_er60_all_classes(v):
    g = gg.er_directed(60, 0.5, 7)
    _check_graph(v, g.n, g.src, g.dst, label="er60")


def test_er1000_count_and_count34(v):
    g = gg.config_graph("er1000")
    G = _check_graph(v, g.n, g.src, g.dst, label="er1000")
    o3, o4 = v.count34(G)
    want3, _ = oracle.count(g.n, g.src, g.dst, 3)
    want4, _ = oracle.count(g.n, g.src, g.dst, 4)
    assert (_np(o3) == want3).all() and (_np(o4) == want4).all()


def test_chunglu_small_full(v):
    """Scaled-down Chung-Lu (same recipe, n = 2,000, 2.5e7 4-sets): hubs, reciprocated arcs."""
    g = gg.config_graph("chunglu_2000")
    _check_graph(v, g.n, g.src, g.dst, label="chunglu_2000")


def test_dense_long_children_rows(v):
    # every vertex has more than 64 neighbours, so every depth-2 child has a long row and
    # the (1,2,0) pairs of children are all tested in the long-vertex bitmap (dozens of
    # long children per slot).  The oracle's rows of a few vertices (its full count of
    # this graph takes minutes), plus the shape totals.
    g = gg.er_directed(300, 0.25, (71, 1))
    _say(f"dense long children n={g.n} m={g.m}")
    G = v.Graph(g.n, g.src, g.dst)
    got = _np(v.count(G, 4))
    rows = np.array([0, 150, 299], np.int32)
    want = oracle.count_rows(g.n, g.src, g.dst, 4, rows)
    assert (got[rows] == want).all()
    sc = v.shape_counts(G)
    assert int(got.sum()) == 4 * (sc["(3,0,0)"] + sc["(2,1,0)"] + sc["(1,2,0)"] + sc["(1,1,1)"])


def test_degenerate_graphs(v):
    import torch
    for n, src, dst in [
        (0, [], []),
        (1, [], []),
        (2, [0], [1]),
        (3, [0, 1], [1, 2]),
        (7, [], []),
        (5, [0, 1, 2], [0, 1, 2]),            # self-loops only
        (9, [0, 1, 2, 3], [1, 0, 3, 2]),      # pairs only: no connected 3-sets
    ]:
        s = np.array(src, np.int32)
        d = np.array(dst, np.int32)
        _check_graph(v, n, s, d, label=f"degenerate n={n}")


def test_errors(v):
    import torch
    g = gg.er_directed(20, 0.2, 1)
    G = v.Graph(g.n, g.src, g.dst)
    out = torch.zeros((20, 199), dtype=torch.int64, device="cuda")
    with pytest.raises(v.VdmcError) as e:
        v.count(G, 5, out)
    assert e.value.name == "UNSUPPORTED"
    with pytest.raises(v.VdmcError) as e:
        v.count(G, 2, out)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(v.VdmcError) as e:
        v.Graph(4, np.array([0, 5], np.int32), np.array([1, 2], np.int32))
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(v.VdmcError):
        v.count(G, 4, torch.zeros((19, 199), dtype=torch.int64, device="cuda"))


def test_relabelling_and_repeat_invariance(v):
    g = gg.er_directed(400, 0.02, 31)
    perm = np.random.default_rng(8).permutation(400).astype(np.int32)
    A = v.Graph(400, g.src, g.dst)
    B = v.Graph(400, perm[g.src], perm[g.dst])
    for k in (3, 4):
        a1 = _np(v.count(A, k))
        a2 = _np(v.count(A, k))
        b = _np(v.count(B, k))
        assert (a1 == a2).all()
        assert (b[perm] == a1).all()


def test_count_range_slices_sum_to_count(v):
    """Root-rank ranges are independent (Lemma 1): consecutive ranges accumulate to the
    full count, for both the light-root and the hub path."""
    import torch
    g = gg.config_graph("chunglu_2000")
    G = v.Graph(g.n, g.src, g.dst)
    for k in (3, 4):
        full = _np(v.count(G, k)).copy()
        out = torch.empty((g.n, v.num_classes(k)), dtype=torch.int64, device="cuda")
        bounds = [0, 1, 7, 64, 300, 1999, g.n]
        for i in range(len(bounds) - 1):
            v.count_range(G, k, out, bounds[i], bounds[i + 1], accumulate=i > 0)
        assert (_np(out) == full).all()
        with pytest.raises(v.VdmcError):
            v.count_range(G, k, out, 5, 2, accumulate=False)


# --------------------------------------------------------------------------- diagnostics

def test_kernel_times_and_hub_share(v):
    # the per-kernel event times and the hub kernel's share of the shape counts
    g = gg.config_graph("chunglu_2000")
    _say(f"kernel times n={g.n}")
    G = v.Graph(g.n, g.src, g.dst)
    v.count34(G)
    light_ms, hub_ms, khub_ms = v.kernel_times(G)
    pc = v.profile_counters(G)
    all_hub = os.environ.get("VDMC_HUB_MIN") == "1"   # every root on the hub path
    assert hub_ms >= 0.0 and (light_ms == -1.0 if all_hub else light_ms >= 0.0)
    assert 0.0 <= khub_ms <= hub_ms   # the hub kernel is the first part of the hub path
    assert all(pc[32 + s] <= pc[s] for s in range(6))
    assert pc[32:38].sum() > 0   # chunglu_2000 has hub roots
    G2 = v.Graph(5, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    v.count(G2, 3)
    lt, ht, kt = v.kernel_times(G2)
    if all_hub:
        assert lt == -1.0 and ht >= 0.0 and kt >= 0.0
    else:
        assert ht == -1.0 and kt == -1.0 and lt >= 0.0   # no hub root: no hub path


# --------------------------------------------------------------------------- undirected motifs

def _undirected_cases():
    star_clique_s = [0] * 9 + [10 + i for i in range(6) for j in range(6) if i < j]
    star_clique_d = list(range(1, 10)) + [10 + j for i in range(6) for j in range(6) if i < j]
    return {
        "er60_dense": gg.er_directed(60, 0.3, (81, 1)),
        "er200": gg.er_directed(200, 0.03, (81, 2)),
        "chunglu_2000": gg.config_graph("chunglu_2000"),
        "star_and_clique": gg.Graph(16, np.array(star_clique_s, np.int32), np.array(star_clique_d, np.int32), "sc"),
    }


@pytest.mark.parametrize("case", ["er60_dense", "er200", "chunglu_2000", "star_and_clique"])
def test_undirected_parity(v, case):
    g = _undirected_cases()[case]
    _say(f"undirected case {case} n={g.n} m={g.m}")
    G = v.Graph(g.n, g.src, g.dst, undirected=True)
    for k in (3, 4):
        assert (v.undirected_classes(k) == oracle.undirected_classes(k)).all()
        got = _np(v.count_undirected(G, k))
        want, _ = oracle.count_undirected(g.n, g.src, g.dst, k)
        assert got.shape == want.shape
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{case} k={k}: {bad.shape[0]} cells differ, first {bad[:5].tolist()}"


def test_undirected_graph_counts_the_symmetric_digraph(v):
    # a graph built with the undirected flag is the digraph with every arc reciprocated
    g = gg.er_directed(120, 0.05, (81, 3))
    G = v.Graph(g.n, g.src, g.dst, undirected=True)
    s2 = np.concatenate([g.src, g.dst])
    d2 = np.concatenate([g.dst, g.src])
    for k in (3, 4):
        want, _ = oracle.count(g.n, s2, d2, k)
        assert (_np(v.count(G, k)) == want).all()


def test_undirected_errors(v):
    g = gg.er_directed(30, 0.1, (81, 4))
    G = v.Graph(g.n, g.src, g.dst)
    with pytest.raises(v.VdmcError) as e:
        v.count_undirected(G, 3)
    assert e.value.name == "INVALID_ARG"
    Gu = v.Graph(g.n, g.src, g.dst, undirected=True)
    with pytest.raises(v.VdmcError) as e:
        v.count_undirected(Gu, 5)
    assert e.value.name in ("UNSUPPORTED", "INVALID_ARG")
    G0 = v.Graph(0, np.zeros(0, np.int32), np.zeros(0, np.int32), undirected=True)
    assert v.count_undirected(G0, 4).shape == (0, 6)


# --------------------------------------------------------------------------- per-edge counts

@pytest.mark.parametrize("case", ["er60_dense", "er200", "chunglu_2000", "star_and_clique"])
def test_edge_parity(v, case):
    g = _undirected_cases()[case]
    _say(f"per-edge case {case} n={g.n} m={g.m}")
    G = v.Graph(g.n, g.src, g.dst)
    lo, hi = v.edge_list(G)
    for k in (3, 4):
        olo, ohi, want = oracle.count_edges(g.n, g.src, g.dst, k)
        assert (lo == olo).all() and (hi == ohi).all()
        got = _np(v.count_edges(G, k))
        assert got.shape == want.shape
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{case} k={k}: {bad.shape[0]} cells differ, first {bad[:5].tolist()}"


def test_edge_counts_edge_cases(v):
    G0 = v.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert v.count_edges(G0, 4).shape == (0, 199)
    assert v.edge_list(G0)[0].shape == (0,)
    G1 = v.Graph(3, np.array([0, 1, 1], np.int32), np.array([1, 0, 2], np.int32))   # one reciprocal pair
    got = _np(v.count_edges(G1, 3))
    olo, ohi, want = oracle.count_edges(3, np.array([0, 1, 1]), np.array([1, 0, 2]), 3)
    assert (got == want).all() and got.sum() == 2
    with pytest.raises(v.VdmcError) as e:
        v.count_edges(G1, 5)
    assert e.value.name in ("UNSUPPORTED", "INVALID_ARG")
