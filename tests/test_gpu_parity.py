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


PATHS = ["default", "hub"]   # "hub": every root with a higher neighbour takes the hub path


def _check_graph(v, n, src, dst, ks=(3, 4), threads=None, label="", path="default"):
    _say(f"case {label} n={n} m={len(src)} path={path}")
    G = v.Graph(n, src, dst)
    if path == "hub":
        v.set_hub_threshold(G, 1)
    for k in ks:
        got = _np(v.count(G, k))
        want, tot = oracle.count(n, src, dst, k, threads=threads)
        assert got.shape == want.shape
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{label} k={k}: {bad.shape[0]} cells differ, first {bad[:5].tolist()}"
        sc = v.shape_counts(G)   # sets visited one by one, per shape
        if k == 3:
            assert sc["(1,1)"] + sc["(1,2)"] == int(tot.sum())
        else:
            assert sc["(3,0,0)"] + sc["(2,1,0)"] + sc["(1,2,0)"] + sc["(1,1,1)"] == int(tot.sum())
    if tuple(ks) == (3, 4):
        o3, o4 = v.count34(G)
        want3, _ = oracle.count(n, src, dst, 3, threads=threads)
        want4, _ = oracle.count(n, src, dst, 4, threads=threads)
        assert (_np(o3) == want3).all() and (_np(o4) == want4).all(), f"{label}: count34 differs"
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

@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(16))
def test_tiny_random_graphs(v, seed, path):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 14))
    p = float(rng.uniform(0.05, 0.8))
    g = gg.er_directed(n, p, (21, seed))
    _check_graph(v, n, g.src, g.dst, label=f"tiny{seed}", path=path)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("kind", ["complete", "tournament", "cycle", "outstar", "instar", "path"])
def test_special_graphs(v, kind, path):
    n = 12
    g = gg.special_graph(kind, n)
    _check_graph(v, n, g.src, g.dst, label=kind, path=path)


@pytest.mark.parametrize("path", PATHS)
def test_dense_er60_all_classes(v, path):
    g = gg.er_directed(60, 0.5, 7)
    _check_graph(v, g.n, g.src, g.dst, label="er60", path=path)


@pytest.mark.parametrize("path", PATHS)
def test_er1000(v, path):
    g = gg.config_graph("er1000")
    _check_graph(v, g.n, g.src, g.dst, label="er1000", path=path)


@pytest.mark.parametrize("path", PATHS)
def test_chunglu_small_full(v, path):
    """Scaled-down Chung-Lu (same recipe, n = 2,000, 2.5e7 4-sets): hubs, reciprocated arcs."""
    g = gg.config_graph("chunglu_2000")
    _check_graph(v, g.n, g.src, g.dst, label="chunglu_2000", path=path)


@pytest.mark.parametrize("path", PATHS)
def test_dense_long_children(v, path):
    # every vertex has about 150 neighbours: every slot's row above the root is longer
    # than 64 entries, so the (1,2,0)/(1,1,1) sets below it take the long-slot kernel;
    # dense local adjacency among the slots.  Full comparison with the oracle.
    g = gg.er_directed(160, 0.5, (71, 1))
    _check_graph(v, g.n, g.src, g.dst, label="dense160", path=path)


def _hub_graph(d, outer, seed):
    """A root of degree d (rank 0) with random arc directions (some reciprocal), sparse arcs
    among its neighbours, `outer` vertices each joined to a few neighbours (depth-2
    vertices with one or several parents) and sparsely to each other (depth 3), and a few
    neighbours with long rows into the outer vertices."""
    rng = np.random.default_rng(seed)
    n = 1 + d + outer
    leaves = np.arange(1, d + 1)
    outs = np.arange(d + 1, n)
    src, dst = [], []
    kind = rng.integers(0, 3, size=d)
    for x, k in zip(leaves, kind):
        if k in (0, 2):
            src.append(0); dst.append(x)
        if k in (1, 2):
            src.append(x); dst.append(0)
    m_local = 2 * d
    src += list(rng.choice(leaves, m_local)); dst += list(rng.choice(leaves, m_local))
    for o in outs:
        for x in rng.choice(leaves, int(rng.integers(1, 5)), replace=False):
            if rng.random() < 0.5:
                src.append(o); dst.append(x)
            else:
                src.append(x); dst.append(o)
    src += list(rng.choice(outs, 2 * outer)); dst += list(rng.choice(outs, 2 * outer))
    for x in rng.choice(leaves, 4, replace=False):   # long rows below the root
        for o in rng.choice(outs, min(100, outer), replace=False):
            src.append(x); dst.append(o)
    return gg.Graph(n, np.array(src, np.int32), np.array(dst, np.int32), f"hub{d}")


@pytest.mark.parametrize("path", PATHS)
def test_hub_root_over_1024(v, path):
    """One root with 1,100 higher neighbours (a hub root between 1,025 and 2,048), every
    shape below it, counted in full and compared with the oracle."""
    g = _hub_graph(1100, 300, 91)
    G = _check_graph(v, g.n, g.src, g.dst, label="hub1100", path=path)
    assert G.max_deg >= 1100


def test_heavy_hubs_shared_by_workgroups(v):
    """A serving-pool graph whose work sits in a few heavy hub roots (n = 5624, largest
    degree 1144): under the default hub threshold its heaviest roots exceed the device's
    fair share and are each taken by several workgroups (every task of such a root by
    exactly one of them); every row equals the oracle's, k = 3 and k = 4."""
    g = gg.serve_pool(70, 2.0, 4.5, 2.0, 10.0, seed=5)[69]
    assert g.n == 5624
    _check_graph(v, g.n, g.src, g.dst, ks=(3,), label="serve pool[69]")
    _check_graph(v, g.n, g.src, g.dst, ks=(4,), label="serve pool[69]")


def test_root_over_2048_takes_per_root_kernel(v):
    """A root with 2,100 higher neighbours (more than the hub path stages) goes through the
    per-root kernel: k = 3 in full against the oracle; k = 4 against the closed form of an
    out-star (centre C(2099+1, 3) sets, each leaf C(2099, 2), one class) and the oracle's
    rows of a few leaves."""
    from math import comb
    n = 2101
    g = gg.special_graph("outstar", n)
    G = _check_graph(v, n, g.src, g.dst, ks=(3,), label="outstar2101")
    got = _np(v.count(G, 4))
    cls0 = 0   # the out-star class (canonical index 7) has class id 0
    assert got[0, cls0] == comb(n - 1, 3) and got[0].sum() == comb(n - 1, 3)
    assert (got[1:, cls0] == comb(n - 2, 2)).all() and int(got[1:].sum()) == (n - 1) * comb(n - 2, 2)
    rows = np.array([1, 1050, 2100], np.int32)
    assert (got[rows] == oracle.count_rows(n, g.src, g.dst, 4, rows)).all()
    # the same star with sparse arcs among the leaves, k = 3 in full
    rng = np.random.default_rng(5)
    s2 = np.concatenate([g.src, rng.integers(1, n, 3000).astype(np.int32)])
    d2 = np.concatenate([g.dst, rng.integers(1, n, 3000).astype(np.int32)])
    _check_graph(v, n, s2, d2, ks=(3,), label="outstar2101+leaf arcs")


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
        for path in PATHS:
            _check_graph(v, n, s, d, label=f"degenerate n={n}", path=path)


def test_errors(v):
    import torch
    g = gg.er_directed(20, 0.2, 1)
    G = v.Graph(g.n, g.src, g.dst)
    out = torch.zeros((20, 199), dtype=torch.int64, device="cuda")
    with pytest.raises(v.VdmcError) as e:
        v.count(G, 6, out)
    assert e.value.name == "INVALID_ARG"
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


@pytest.mark.parametrize("path", PATHS)
def test_count_range_slices_sum_to_count(v, path):
    """Root-rank ranges are independent (Lemma 1): consecutive ranges accumulate to the
    full count, for both the light-root and the hub path."""
    import torch
    g = gg.config_graph("chunglu_2000")
    G = v.Graph(g.n, g.src, g.dst)
    if path == "hub":
        v.set_hub_threshold(G, 1)
    for k in (3, 4):
        want, _ = oracle.count(g.n, g.src, g.dst, k)
        out = torch.empty((g.n, v.num_classes(k)), dtype=torch.int64, device="cuda")
        bounds = [0, 1, 7, 64, 300, 1999, g.n]
        for i in range(len(bounds) - 1):
            v.count_range(G, k, out, bounds[i], bounds[i + 1], accumulate=i > 0)
        assert (_np(out) == want).all()
        with pytest.raises(v.VdmcError):
            v.count_range(G, k, out, 5, 2, accumulate=False)


def test_hub_threshold_changes_nothing(v):
    g = gg.config_graph("chunglu_2000")
    G = v.Graph(g.n, g.src, g.dst)
    want, _ = oracle.count(g.n, g.src, g.dst, 4)
    for t in (1, 2, 8, 32, 100, 1 << 30):
        v.set_hub_threshold(G, t)
        assert (_np(v.count(G, 4)) == want).all(), f"threshold {t}"
    with pytest.raises(v.VdmcError) as e:
        v.set_hub_threshold(G, 0)
    assert e.value.name == "INVALID_ARG"


# --------------------------------------------------------------------------- diagnostics

def test_kernel_times(v):
    g = gg.config_graph("chunglu_2000")
    _say(f"kernel times n={g.n}")
    G = v.Graph(g.n, g.src, g.dst)
    v.count34(G)
    light_ms, hub_ms, khub_ms = v.kernel_times(G)
    assert hub_ms >= 0.0 and light_ms >= 0.0
    assert 0.0 <= khub_ms <= hub_ms   # the hub kernel is the first part of the hub path
    G2 = v.Graph(5, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    v.count(G2, 3)
    lt, ht, kt = v.kernel_times(G2)
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
