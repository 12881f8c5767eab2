"""Sec. 7 at the paper's own scale, on the GPU path: G(n = 1000, p = 1/10), directed and
undirected, k = 3 and 4.  Eq. 4 summed over the vertices (each set once): the expected
number of sets of class m is C(n, k) N_Iso(m) p^e(m) (1 - p)^(L - e(m)), L = k(k-1) arcs
(directed) or C(k, 2) edges (undirected), N_Iso(m) = number of labelled graphs in the
class, e(m) = its arcs or edges.  Over R seeded graphs, the mean count of every class
with an expectation of at least 10 must lie within a t-test bound of it, family-wise
level 1% over the classes (Bonferroni; the paper reports a non-significant chi-square
for every motif at n = 1000; the standard error here is measured across the seeds).  The oracle is too slow at this size; this checks
the HIP path against the theory directly."""
import itertools
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
import oracle.exhaustive as ex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def v():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_11655_amd as v
    v.load()
    return v


def _directed_theory(k):
    _, cls, codes = oracle.class_table(k)
    C = len(codes)
    n_iso, e = np.zeros(C), np.zeros(C)
    for code in range(1 << (k * (k - 1))):
        if cls[code] >= 0:
            n_iso[cls[code]] += 1
            e[cls[code]] = bin(code).count("1")
    return n_iso, e, k * (k - 1)


def _undirected_theory(k):
    # columns in the order of oracle.undirected_classes, named from their codes
    _, _, codes = oracle.class_table(k)
    names = []
    for c in oracle.undirected_classes(k):
        A = ex.matrix_of(k, int(codes[c]))
        names.append(ex.undirected_name(k, [(i, j) for i in range(k) for j in range(i + 1, k) if A[i][j]]))
    pairs = list(itertools.combinations(range(k), 2))
    n_iso, e = np.zeros(len(names)), np.zeros(len(names))
    for mask in range(1 << len(pairs)):
        edges = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
        seen, stack = {0}, [0]
        while stack:
            x = stack.pop()
            for i, j in edges:
                y = j if i == x else (i if j == x else None)
                if y is not None and y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) < k:
            continue
        j = names.index(ex.undirected_name(k, edges))
        n_iso[j] += 1
        e[j] = len(edges)
    return n_iso, e, len(pairs)


@pytest.mark.parametrize("k", [3, 4])
@pytest.mark.parametrize("directed", [True, False])
def test_er_expectation_paper_scale(v, k, directed):
    import torch
    from scipy import stats
    n, p, R = 1000, 0.1, 16
    n_iso, e, L = _directed_theory(k) if directed else _undirected_theory(k)
    expect = math.comb(n, k) * n_iso * p ** e * (1 - p) ** (L - e)
    samples = []
    for r in range(R):
        print(f"G(1000, 0.1) directed={directed} k={k} seed {r}", flush=True)
        g = (gg.er_directed if directed else gg.er_undirected)(n, p, (91, k, int(directed), r))
        G = v.Graph(n, g.src, g.dst, undirected=not directed)
        out = v.count(G, k) if directed else v.count_undirected(G, k)
        col = out.sum(dim=0).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        assert np.all(np.mod(col, k) == 0)
        samples.append(col / k)
    S = np.array(samples)
    mean, sd = S.mean(axis=0), S.std(axis=0, ddof=1)
    big = expect >= 10
    assert big.sum() >= (len(expect) - 2 if directed else len(expect))
    se = np.maximum(sd[big], 1.0) / math.sqrt(R)
    z = np.abs(mean[big] - expect[big]) / se
    bound = stats.t.ppf(1.0 - 0.005 / big.sum(), R - 1)
    print(f"max |t| over {big.sum()} classes: {z.max():.2f} (bound {bound:.2f})", flush=True)
    assert (z < bound).all()
