"""Input generators: determinism and the stated structure of each recipe."""
import numpy as np

import graphgen as gg


def _und_degree(g):
    s = g.src.astype(np.int64)
    d = g.dst.astype(np.int64)
    lo, hi = np.minimum(s, d), np.maximum(s, d)
    pk = np.unique(lo * g.n + hi)
    return np.bincount(np.concatenate([pk // g.n, pk % g.n]), minlength=g.n)


def test_seeded_and_repeatable():
    a = gg.er_directed(300, 0.02, (1, 2))
    b = gg.er_directed(300, 0.02, (1, 2))
    assert gg.digest(a) == gg.digest(b)
    assert gg.digest(a) != gg.digest(gg.er_directed(300, 0.02, (1, 3)))


def test_keyed_cap_bounds_every_undirected_degree():
    g = gg.rmat(12, 8, 0.57, 0.19, 0.19, 20, 9)
    deg = _und_degree(g)
    assert deg.max() <= 20
    assert (g.src != g.dst).all()
    assert np.unique(g.src.astype(np.int64) * g.n + g.dst).shape[0] == g.m   # no repeated arcs


def test_chung_lu_reciprocation_and_cap():
    g = gg.chung_lu(20000, 100000, 2.1, 50.0, 0.2, 60, 3)
    assert _und_degree(g).max() <= 60
    arcs = set(zip(g.src.tolist(), g.dst.tolist()))
    recip = sum((b, a) in arcs for a, b in arcs) / len(arcs)
    assert 0.2 < recip < 0.5   # 20% of base arcs reversed -> about a third of arcs in mutual pairs


def test_er_density():
    g = gg.er_directed(1000, 0.005, 1)
    assert abs(g.m - 0.005 * 1000 * 999) < 5 * np.sqrt(0.005 * 1000 * 999)
    assert (g.src != g.dst).all()
