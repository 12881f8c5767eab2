"""Pins of the CPU oracle to facts outside itself (no GPU needed).

Each test names the passage or the mathematical fact it rests on.  A plausible slip in
the oracle -- a transposed adjacency entry, a wrong bit order, a missed connected set,
a double count, a crediting error -- fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
import oracle.exhaustive as ex

from conftest import read_golden


# --------------------------------------------------------------------------- encoding

def test_fig1_index_and_minimal_index():
    """Sec. 4.1, Fig. 1: the printed matrix reads 110101 = 53; its minimal isomorph is 30."""
    rows = read_golden("fig1_index.txt")
    k = int(dict(rows)["k"][0])
    A = [[int(x) for x in v] for key, v in rows if key == "row"]
    vals = {key: v[0] for key, v in rows if key != "row"}
    bits = "".join(str(A[i][j]) for i in range(k) for j in range(k) if i != j)
    assert bits == vals["bitstring"]
    assert ex.motif_index(A) == int(vals["index"]) == int(vals["bitstring"], 2)
    assert ex.minimal_index(k, int(vals["index"])) == int(vals["min_index"])
    canon, cls, codes = oracle.class_table(k)
    assert canon[int(vals["index"])] == int(vals["min_index"])
    # the isomorph the paper names (30 = 011110) is a relabelling of the same motif
    assert canon[30] == 30 and cls[53] == cls[30] >= 0


@pytest.mark.parametrize("k", [3, 4, 5])
def test_class_table_sizes_match_known_enumerations(k):
    """Sizes of the class tables equal the textbook digraph counts (golden file)."""
    ref = {}
    for key, v in read_golden("digraph_counts.txt"):
        d = dict(zip(v[1::2], v[2::2]))
        ref[int(v[0])] = {kk: int(x) for kk, x in d.items()}
    canon, cls, codes = oracle.class_table(k)
    assert len(np.unique(canon)) == ref[k]["all"]
    assert len(codes) == ref[k]["connected"] == oracle.NUM_CLASSES[k]
    assert int((cls >= 0).sum()) == ref[k]["labelled_connected"]
    if k <= 4:
        # pure-Python table built independently agrees code by code
        mins, conn = ex.classes(k)
        assert list(codes) == conn
        assert list(canon) == mins
    else:
        # 2^20 codes are too many for the pure-Python table: a seeded sample of codes, plus
        # every class representative, checked against it one by one
        rng = np.random.default_rng(55)
        sample = set(rng.integers(0, 1 << 20, 600).tolist()) | set(codes[::97].tolist())
        for c in sorted(sample):
            assert canon[c] == ex.minimal_index(k, c)
            assert (cls[c] >= 0) == ex.weakly_connected(ex.matrix_of(k, c))
    # class ids ascend with the canonical code and every code maps to its own class
    assert all(codes[i] < codes[i + 1] for i in range(len(codes) - 1))
    for c in range(1 << (k * (k - 1))):
        if cls[c] >= 0:
            assert codes[cls[c]] == canon[c]


def _pairs_and_reciprocal(k, code):
    A = np.array(ex.matrix_of(k, code), dtype=int)
    U = (A + A.T) > 0
    return int(U.sum() // 2), int(((A + A.T) == 2).sum() // 2)


def test_sparse_class_families():
    """The class families the whole-graph kernels keep LDS counters for, counted in the
    oracle's tables against counts fixed independently:
    - classes whose underlying graph is a tree with single arcs = oriented trees on k
      nodes, OEIS A000238 (1, 1, 3, 8, 27, ...): 3, 8, 27 for k = 3, 4, 5;
    - k = 4 trees with any arc states: 3-stars are multisets of 3 leaf arcs over 3 states,
      C(5, 3) = 10; 4-paths are arc triples up to reversal (which swaps each arc's
      direction), (27 + 3) / 2 = 15 by Burnside; 25 in all;
    - k = 4 classes with four joined pairs, all single arcs: oriented 4-cycles (4) and
      oriented tailed triangles (2^4 / 2 = 8: the swap of the two unattached triangle
      vertices reverses their arc, so it fixes no orientation); 12 in all."""
    fam = {}
    for k in (3, 4, 5):
        _, _, codes = oracle.class_table(k)
        pr = [_pairs_and_reciprocal(k, int(c)) for c in codes]
        fam[k] = {
            "single_arc_trees": sum(1 for e, r in pr if e == k - 1 and r == 0),
            "trees": sum(1 for e, r in pr if e == k - 1),
            "single_arc_4pair": sum(1 for e, r in pr if e == 4 and r == 0),
        }
    assert [fam[k]["single_arc_trees"] for k in (3, 4, 5)] == [3, 8, 27]
    assert fam[4]["trees"] == 25
    assert fam[4]["single_arc_4pair"] == 12


def test_k3_class_structure_by_hand():
    """The 13 connected 3-vertex digraphs by number of arcs, counted by hand:
    2 arcs: out-star, in-star, path (3); 3 arcs: cycle, transitive triangle, a mutual
    pair plus an arc out of or into the third vertex... (4); 4 arcs: 4; 5 arcs: 1;
    6 arcs: the complete digraph (1)."""
    canon, cls, codes = oracle.class_table(3)
    per_e = {}
    for c in codes:
        e = bin(int(c)).count("1")
        per_e[e] = per_e.get(e, 0) + 1
    assert per_e == {2: 3, 3: 4, 4: 4, 5: 1, 6: 1}


# --------------------------------------------------------------------------- CSR example

def test_csr_example_of_sec42():
    """Sec. 4.2: the example graph's undirected CSR (Indices/Neighbors) and, restricted to
    out-arcs, its directed CSR."""
    rows = read_golden("csr_example.txt")
    d = {}
    arcs = []
    for key, v in rows:
        if key == "arc":
            arcs.append((int(v[0]), int(v[1])))
        else:
            d[key] = [int(x) for x in v]
    n = d["n"][0]
    src = np.array([a for a, _ in arcs], np.int32)
    dst = np.array([b for _, b in arcs], np.int32)
    off, nbr, dr = oracle.simple_graph(n, src, dst)
    assert off.tolist() == d["undirected_indices"]
    assert nbr.tolist() == d["undirected_neighbors"]
    out_idx = [0]
    out_nbr = []
    for v in range(n):
        for e in range(off[v], off[v + 1]):
            if dr[e] & 1:
                out_nbr.append(int(nbr[e]))
        out_idx.append(len(out_nbr))
    assert out_idx == d["directed_indices"]
    assert out_nbr == d["directed_neighbors"]


def test_csr_example_motifs():
    """Motifs of the Sec. 4.2 example graph, derived by hand from its four arcs sets:
    the four 3-sets are all connected, the one 4-set is connected."""
    src = np.array([0, 0, 0, 2, 3, 3], np.int32)
    dst = np.array([1, 2, 3, 0, 1, 2], np.int32)
    c3, t3 = oracle.count(4, src, dst, 3, threads=1)
    assert int(t3.sum()) == 4 and (c3.sum(axis=1) == 3).all()
    c4, t4 = oracle.count(4, src, dst, 4, threads=1)
    assert int(t4.sum()) == 1 and (c4.sum(axis=1) == 1).all()
    # {0,1,2,3} has arcs 0->1 0->2 0->3 2->0 3->1 3->2: its minimal index by brute force
    A = [[0] * 4 for _ in range(4)]
    for a, b in zip(src, dst):
        A[a][b] = 1
    _, _, codes = oracle.class_table(4)
    want = ex.minimal_index(4, ex.motif_index(A))
    assert codes[np.nonzero(c4[0])[0][0]] == want


# --------------------------------------------------------------------------- closed forms

def _class_of_matrix(k, A):
    _, _, codes = oracle.class_table(k)
    return list(codes).index(ex.minimal_index(k, ex.motif_index(A)))


@pytest.mark.parametrize("k", [3, 4, 5])
def test_complete_bidirected(k):
    """K_n with every ordered pair an arc: every k-set is the complete motif, so each
    vertex lies in C(n-1, k-1) of them (cliques: Sec. 7 validation on toy graphs)."""
    n = 9
    g = gg.special_graph("complete", n)
    c, t = oracle.count(n, g.src, g.dst, k, threads=2)
    cid = _class_of_matrix(k, [[int(i != j) for j in range(k)] for i in range(k)])
    assert cid == oracle.NUM_CLASSES[k] - 1   # the all-ones code is the largest
    assert (c[:, cid] == math.comb(n - 1, k - 1)).all()
    assert int(c.sum()) == n * math.comb(n - 1, k - 1)
    assert int(t[cid]) == math.comb(n, k)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_transitive_tournament(k):
    """Regular DAG i -> j for i < j: every k-set induces the transitive tournament."""
    n = 10
    g = gg.special_graph("tournament", n)
    c, _ = oracle.count(n, g.src, g.dst, k, threads=2)
    cid = _class_of_matrix(k, [[int(i < j) for j in range(k)] for i in range(k)])
    assert (c[:, cid] == math.comb(n - 1, k - 1)).all()
    assert int(c.sum()) == n * math.comb(n - 1, k - 1)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_directed_cycle(k):
    """Directed n-cycle (n > k): the connected k-sets are the n windows of k consecutive
    vertices, each a directed path; every vertex lies in k of them."""
    n = 11
    g = gg.special_graph("cycle", n)
    c, t = oracle.count(n, g.src, g.dst, k, threads=2)
    cid = _class_of_matrix(k, [[int(j == i + 1) for j in range(k)] for i in range(k)])
    assert (c[:, cid] == k).all() and int(c.sum()) == n * k and int(t.sum()) == n


@pytest.mark.parametrize("k", [3, 4, 5])
def test_k_cycle_alone(k):
    """A directed k-cycle on k vertices is one motif; each vertex gets one count."""
    g = gg.special_graph("cycle", k)
    c, t = oracle.count(k, g.src, g.dst, k, threads=1)
    cid = _class_of_matrix(k, [[int(j == (i + 1) % k) for j in range(k)] for i in range(k)])
    assert (c[:, cid] == 1).all() and int(c.sum()) == k


@pytest.mark.parametrize("k", [3, 4, 5])
@pytest.mark.parametrize("kind", ["outstar", "instar"])
def test_stars(k, kind):
    """Star with hub 0: the hub lies in C(n-1, k-1) sets, every leaf in C(n-2, k-2)."""
    n = 10
    g = gg.special_graph(kind, n)
    c, _ = oracle.count(n, g.src, g.dst, k, threads=2)
    if kind == "outstar":
        A = [[int(i == 0 and j > 0) for j in range(k)] for i in range(k)]
    else:
        A = [[int(j == 0 and i > 0) for j in range(k)] for i in range(k)]
    cid = _class_of_matrix(k, A)
    assert int(c[0, cid]) == math.comb(n - 1, k - 1)
    assert (c[1:, cid] == math.comb(n - 2, k - 2)).all()
    assert int(c.sum()) == k * math.comb(n - 1, k - 1)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_degenerate_inputs(k):
    """n < k, no arcs, self-loops only, isolated vertices: all-zero rows."""
    c, t = oracle.count(k - 1, np.array([0], np.int32), np.array([1], np.int32), k, threads=1)
    assert c.sum() == 0 and t.sum() == 0
    c, t = oracle.count(7, np.zeros(0, np.int32), np.zeros(0, np.int32), k, threads=1)
    assert c.sum() == 0
    loops = np.arange(7, dtype=np.int32)
    c, t = oracle.count(7, loops, loops, k, threads=1)
    assert c.sum() == 0
    with pytest.raises(ValueError):
        oracle.count(3, np.array([0], np.int32), np.array([5], np.int32), k)


# --------------------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(12))
def test_esu_equals_brute_force_small(seed):
    """ESU (C) against the plain definition over all k-subsets (pure Python)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 12))
    p = float(rng.uniform(0.1, 0.7))
    g = gg.er_directed(n, p, (11, seed))
    # add duplicates and self-loops: normalisation must ignore them
    src = np.concatenate([g.src, g.src[:3], np.arange(2, dtype=np.int32)])
    dst = np.concatenate([g.dst, g.dst[:3], np.arange(2, dtype=np.int32)])
    for k in (3, 4):
        a, ta = oracle.count(n, src, dst, k, threads=3)
        b, tb = ex.count(n, src, dst, k)
        assert (a == b).all() and (ta == tb).all()


def _by_code(k, c):
    """Oracle per-vertex counts keyed by minimal index, as the brute force keys them."""
    _, _, codes = oracle.class_table(k)
    cols = np.nonzero(c.sum(axis=0))[0]
    return {int(codes[j]): c[:, j] for j in cols}


@pytest.mark.parametrize("seed", range(10))
def test_esu_equals_brute_force_k5(seed):
    """k = 5: ESU (C) against the plain definition over all 5-subsets, compared per
    minimal index (the brute force canonicalises each set it meets by trying all 120
    relabellings, independently of the oracle's table)."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 11))
    p = float(rng.uniform(0.15, 0.6))
    g = gg.er_directed(n, p, (12, seed))
    src = np.concatenate([g.src, g.src[:2], np.arange(2, dtype=np.int32)])
    dst = np.concatenate([g.dst, g.dst[:2], np.arange(2, dtype=np.int32)])
    a, ta = oracle.count(n, src, dst, 5, threads=3)
    rows, tot = ex.count_by_code(n, src, dst, 5)
    got = _by_code(5, a)
    assert sorted(got) == sorted(rows)
    for m in rows:
        assert (got[m] == rows[m]).all()
    _, _, codes = oracle.class_table(5)
    assert {int(codes[j]): int(ta[j]) for j in np.nonzero(ta)[0]} == tot


@pytest.mark.slow
def test_esu_equals_brute_force_dense_all_classes():
    """G(60, 0.5): 487,635 4-subsets, every one of the 199 classes present."""
    g = gg.er_directed(60, 0.5, 7)
    a, ta = oracle.count(60, g.src, g.dst, 4)
    assert (ta > 0).all()
    b, tb = ex.count(60, g.src, g.dst, 4)
    assert (a == b).all() and (ta == tb).all()


def test_invariants_er1000():
    """Column sums are k times the class totals (each set credits its k vertices)."""
    g = gg.config_graph("er1000")
    for k in (3, 4):
        c, t = oracle.count(g.n, g.src, g.dst, k)
        assert (c.sum(axis=0) == k * t).all()
    g = gg.er_directed(300, 0.012, 8)
    c, t = oracle.count(g.n, g.src, g.dst, 5)
    assert (c.sum(axis=0) == 5 * t).all() and t.sum() > 0


def test_relabelling_permutes_rows():
    """Renaming the vertices permutes the rows and changes nothing else."""
    g = gg.er_directed(80, 0.06, 5)
    perm = np.random.default_rng(3).permutation(80).astype(np.int32)
    for k in (3, 4, 5):
        a, _ = oracle.count(80, g.src, g.dst, k)
        b, _ = oracle.count(80, perm[g.src], perm[g.dst], k)
        assert (b[perm] == a).all()


def test_disjoint_union_concatenates():
    g1 = gg.er_directed(30, 0.15, 1)
    g2 = gg.er_directed(25, 0.2, 2)
    src = np.concatenate([g1.src, g2.src + 30])
    dst = np.concatenate([g1.dst, g2.dst + 30])
    for k in (3, 4, 5):
        a, _ = oracle.count(30, g1.src, g1.dst, k)
        b, _ = oracle.count(25, g2.src, g2.dst, k)
        u, _ = oracle.count(55, src, dst, k)
        assert (u[:30] == a).all() and (u[30:] == b).all()


def test_rows_mode_equals_full_rows():
    g = gg.er_directed(150, 0.04, 9)
    rows = np.array([0, 3, 77, 149, 3], np.int32)
    for k in (3, 4, 5):
        full, _ = oracle.count(150, g.src, g.dst, k)
        part = oracle.count_rows(150, g.src, g.dst, k, rows)
        assert (part == full[rows]).all()


# --------------------------------------------------------------------------- Sec. 7

@pytest.mark.parametrize("k", [3, 4, 5])
def test_er_expectation_eq4(k):
    """Sec. 7, Eq. 4 summed over vertices (each set counted once): for directed G(n,p)
    the expected number of sets in class m is C(n,k) N_Iso(m) p^e (1-p)^(k(k-1)-e),
    where N_Iso(m) is the number of labelled codes in the class and e its arc count.
    The mean over R seeds must lie within 5 standard errors for every class with an
    expectation of at least 10."""
    n, p, R = 40, 0.12, 24
    canon, cls, codes = oracle.class_table(k)
    C = len(codes)
    allc = np.arange(1 << (k * (k - 1)), dtype=np.int64)
    conn = cls >= 0
    n_iso = np.bincount(cls[conn], minlength=C).astype(np.float64)
    ones = np.zeros(allc.shape[0], np.int64)
    for b in range(k * (k - 1)):
        ones += (allc >> b) & 1
    e = np.zeros(C)
    e[cls[conn]] = ones[conn]   # relabelling keeps the arc count, so any member will do
    L = k * (k - 1)
    expect = math.comb(n, k) * n_iso * p ** e * (1 - p) ** (L - e)
    samples = []
    for r in range(R):
        g = gg.er_directed(n, p, (7, k, r))
        _, t = oracle.count(n, g.src, g.dst, k)
        samples.append(t.astype(np.float64))
    S = np.array(samples)
    mean = S.mean(axis=0)
    sd = S.std(axis=0, ddof=1)
    big = expect >= 10
    assert big.sum() >= {3: 5, 4: 20, 5: 40}[k]
    se = np.maximum(sd[big], 1.0) / math.sqrt(R)
    assert (np.abs(mean[big] - expect[big]) < 5 * se).all()
    # pooled small classes
    small = ~big
    if small.any():
        pooled = S[:, small].sum(axis=1)
        assert abs(pooled.mean() - expect[small].sum()) < 5 * max(pooled.std(ddof=1), 1.0) / math.sqrt(R) + 1.0


# --------------------------------------------------------------------------- undirected motifs

def _undirected_column_names(k):
    """Name of each undirected column of the oracle, read off its class code."""
    _, _, codes = oracle.class_table(k)
    names = []
    for c in oracle.undirected_classes(k):
        A = ex.matrix_of(k, int(codes[c]))
        edges = [(i, j) for i in range(k) for j in range(i + 1, k) if A[i][j] or A[j][i]]
        assert all(A[i][j] and A[j][i] for i, j in edges)   # every pair reciprocal
        names.append(ex.undirected_name(k, edges))
    return names


@pytest.mark.parametrize("k", [3, 4])
def test_undirected_classes_are_the_connected_graphs(k):
    # Fig. 3 caption: the undirected runs count connected graphs on k vertices: 2 and 6
    names = _undirected_column_names(k)
    assert sorted(names) == sorted(ex.UNDIRECTED_NAMES[k])


def _undirected_by_name(n, src, dst, k):
    got, tot = oracle.count_undirected(n, src, dst, k)
    names = _undirected_column_names(k)
    return {nm: got[:, j] for j, nm in enumerate(names)}, {nm: int(tot[j]) for j, nm in enumerate(names)}


def _edges(pairs):
    s = np.array([a for a, b in pairs], np.int32)
    d = np.array([b for a, b in pairs], np.int32)
    return s, d


def test_undirected_closed_forms():
    comb = math.comb
    # complete graph K7: every vertex in C(6,2) triangles and C(6,3) cliques, nothing else
    n = 7
    s, d = _edges([(i, j) for i in range(n) for j in range(i + 1, n)])
    c3, _ = _undirected_by_name(n, s, d, 3)
    c4, _ = _undirected_by_name(n, s, d, 4)
    assert (c3["triangle"] == comb(6, 2)).all() and (c3["path"] == 0).all()
    assert (c4["clique"] == comb(6, 3)).all() and sum(int(c4[x].sum()) for x in c4 if x != "clique") == 0
    # star with centre 0 and 6 leaves (arcs pointing both ways: directions are ignored)
    s, d = _edges([(0, i) if i % 2 else (i, 0) for i in range(1, 7)])
    c3, _ = _undirected_by_name(7, s, d, 3)
    c4, _ = _undirected_by_name(7, s, d, 4)
    assert c3["path"][0] == comb(6, 2) and (c3["path"][1:] == 5).all()
    assert c4["star"][0] == comb(6, 3) and (c4["star"][1:] == comb(5, 2)).all()
    # path 0-1-2-3-4-5: windows of consecutive vertices
    n = 6
    s, d = _edges([(i, i + 1) for i in range(n - 1)])
    c3, _ = _undirected_by_name(n, s, d, 3)
    c4, _ = _undirected_by_name(n, s, d, 4)
    win = lambda i, w: sum(1 for a in range(0, n - w + 1) if a <= i < a + w)
    assert [int(x) for x in c3["path"]] == [win(i, 3) for i in range(n)]
    assert [int(x) for x in c4["path"]] == [win(i, 4) for i in range(n)]
    # cycle of 6: every vertex on 3 paths of 3 and 4 paths of 4
    s, d = _edges([(i, (i + 1) % n) for i in range(n)])
    c3, _ = _undirected_by_name(n, s, d, 3)
    c4, _ = _undirected_by_name(n, s, d, 4)
    assert (c3["path"] == 3).all() and (c4["path"] == 4).all() and (c4["cycle"] == 0).all()
    # 4-cycle alone, and a diamond (4-cycle plus one chord)
    s, d = _edges([(0, 1), (1, 2), (2, 3), (3, 0)])
    c4, t4 = _undirected_by_name(4, s, d, 4)
    assert t4["cycle"] == 1 and sum(t4.values()) == 1
    s, d = _edges([(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)])
    c4, t4 = _undirected_by_name(4, s, d, 4)
    assert t4["diamond"] == 1 and sum(t4.values()) == 1


@pytest.mark.parametrize("seed", range(6))
def test_undirected_equals_brute_force(seed):
    g = gg.er_directed(11, 0.22, (41, seed))
    for k in (3, 4):
        got, _ = _undirected_by_name(g.n, g.src, g.dst, k)
        want = ex.count_undirected(g.n, g.src, g.dst, k)
        for nm in ex.UNDIRECTED_NAMES[k]:
            assert (got[nm] == want[nm]).all(), (k, nm)


# --------------------------------------------------------------------------- per-edge counts

@pytest.mark.parametrize("seed", range(5))
def test_edge_counts_equal_brute_force(seed):
    g = gg.er_directed(10, 0.25, (43, seed))
    for k in (3, 4):
        lo, hi, got = oracle.count_edges(g.n, g.src, g.dst, k)
        pairs, want = ex.count_edges(g.n, g.src, g.dst, k)
        assert list(zip(lo.tolist(), hi.tolist())) == pairs
        assert (got == want).all()


@pytest.mark.parametrize("k", [3, 4])
def test_edge_counts_closed_forms_and_invariant(k):
    comb = math.comb
    # complete bidirected graph K6: every edge lies in C(4, k-2) sets, all of the last class
    n = 6
    s = np.array([i for i in range(n) for j in range(n) if i != j], np.int32)
    d = np.array([j for i in range(n) for j in range(n) if i != j], np.int32)
    lo, hi, got = oracle.count_edges(n, s, d, k)
    assert len(lo) == comb(n, 2)
    assert (got[:, -1] == comb(n - 2, k - 2)).all() and got[:, :-1].sum() == 0
    # any graph: summing a class's edge counts gives (edges of the class) x (its sets)
    g = gg.er_directed(40, 0.1, (44, k))
    lo, hi, got = oracle.count_edges(g.n, g.src, g.dst, k)
    _, tot = oracle.count(g.n, g.src, g.dst, k)
    _, _, codes = oracle.class_table(k)
    for c in range(len(codes)):
        A = ex.matrix_of(k, int(codes[c]))
        ne = sum(1 for i in range(k) for j in range(i + 1, k) if A[i][j] or A[j][i])
        assert int(got[:, c].sum()) == ne * int(tot[c])
