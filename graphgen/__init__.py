"""Seeded synthetic directed-graph generators.

This module only draws random arc lists.  It holds none of the motif-counting
arithmetic (no adjacency codes, no isomorphism classes, no enumeration), so that
both the CPU oracle's tests and the GPU path can take their inputs from it
without sharing any of the method's code.

Every generator returns ``(n, src, dst)``: the vertex count and two ``int32``
arrays of equal length holding the arcs ``src[i] -> dst[i]`` with ids in
``[0, n)``.  The arc list may contain self-loops and duplicates unless the
recipe says otherwise; the method's input normalisation (the paper works on a
simple graph, Sec. 4.1) is the consumer's job.

Recipes (workloads of the paper: G(n,p) graphs of Sec. 7-8, and synthetic
stand-ins for the fat-tailed real graphs of Sec. 9, Table 1):

* ``er_directed``      -- each ordered pair u != v is an arc with probability p.
* ``chung_lu``         -- power-law expected degrees, independent in/out
                          weights, a reciprocated fraction, keyed degree cap.
* ``rmat``             -- recursive-matrix generator with quadrant probabilities
                          (a, b, c, d), duplicates and self-loops removed,
                          keyed degree cap.
* ``er_batch``         -- many small directed G(n,p) graphs of uneven size.
* ``serve_pool``       -- a pool of resident graphs with log-uniform sizes.

All randomness comes from numpy's PCG64 through ``numpy.random.default_rng``
seeded with the given seed (an int or a tuple of ints).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Graph",
    "er_directed",
    "chung_lu",
    "rmat",
    "keyed_cap",
    "er_batch",
    "serve_pool",
    "config_graph",
    "special_graph",
    "digest",
]


@dataclass
class Graph:
    """An arc list: ``n`` vertices and arcs ``src[i] -> dst[i]``."""

    n: int
    src: np.ndarray
    dst: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _rng(seed):
    if isinstance(seed, (tuple, list)):
        return np.random.default_rng([int(s) for s in seed])
    return np.random.default_rng(int(seed))


def digest(g: Graph) -> str:
    """SHA-256 over (n, src, dst) so that two consumers can prove they saw the same input."""
    h = hashlib.sha256()
    h.update(np.int64(g.n).tobytes())
    h.update(np.ascontiguousarray(g.src, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(g.dst, dtype=np.int32).tobytes())
    return h.hexdigest()


def er_undirected(n: int, p: float, seed) -> Graph:
    """Undirected G(n,p): every unordered pair {u < v} is an edge independently with prob. p,
    emitted as one arc u -> v (directions are to be ignored by the consumer)."""
    rng = _rng(seed)
    n = int(n)
    if n <= 1 or p <= 0.0:
        z = np.zeros(0, np.int32)
        return Graph(n, z, z.copy(), f"er_u({n},{p})")
    mask = np.triu(rng.random((n, n)) < p, 1)
    s, d = np.nonzero(mask)
    return Graph(n, s.astype(np.int32), d.astype(np.int32), f"er_u({n},{p})")


def er_directed(n: int, p: float, seed) -> Graph:
    """Directed G(n,p): every ordered pair (u, v), u != v, is an arc independently with prob. p."""
    rng = _rng(seed)
    n = int(n)
    if n <= 1 or p <= 0.0:
        z = np.zeros(0, np.int32)
        return Graph(n, z, z.copy(), f"er({n},{p})")
    total = n * (n - 1)
    if total <= 4_000_000:
        mask = rng.random((n, n)) < p
        np.fill_diagonal(mask, False)
        s, d = np.nonzero(mask)
    else:
        # Same law without an n x n matrix: the number of arcs is Binomial(n(n-1), p)
        # and, given that number, the arc set is a uniform subset of the ordered pairs.
        m = int(rng.binomial(total, p))
        picked = np.unique(rng.integers(0, total, size=int(m * 1.1) + 16, dtype=np.int64))
        while picked.shape[0] < m:
            more = rng.integers(0, total, size=m, dtype=np.int64)
            picked = np.unique(np.concatenate([picked, more]))
        picked = rng.permutation(picked)[:m]
        picked.sort()
        s = picked // (n - 1)
        r = picked % (n - 1)
        d = r + (r >= s)
    return Graph(n, s.astype(np.int32), d.astype(np.int32), f"er({n},{p})")


def keyed_cap(n: int, src: np.ndarray, dst: np.ndarray, cap: int, seed) -> tuple[np.ndarray, np.ndarray]:
    """Drop self-loops and duplicate arcs, then cap every vertex's undirected degree.

    Each undirected pair gets a seeded uniform key.  At each endpoint the incident pairs
    are ranked by key; a pair (both of its arcs) is kept iff its rank is below ``cap`` at
    both endpoints.  Every remaining undirected degree is then at most ``cap``.
    """
    rng = _rng(seed)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    arc_key = np.unique(src * n + dst)
    src, dst = arc_key // n, arc_key % n
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    pair_key, pair_of_arc = np.unique(lo * n + hi, return_inverse=True)
    npairs = pair_key.shape[0]
    key = rng.random(npairs)
    plo = pair_key // n
    phi = pair_key % n
    # every pair is incident to two vertices; rank all incidences of a vertex together
    end = np.concatenate([plo, phi])
    pidx = np.concatenate([np.arange(npairs), np.arange(npairs)])
    order = np.lexsort((np.concatenate([key, key]), end))
    e_sorted = end[order]
    starts = np.flatnonzero(np.r_[True, e_sorted[1:] != e_sorted[:-1]])
    group_start = np.repeat(starts, np.diff(np.r_[starts, e_sorted.shape[0]]))
    rank_in_group = np.arange(e_sorted.shape[0]) - group_start
    ok = np.ones(npairs, bool)
    ok[pidx[order[rank_in_group >= cap]]] = False
    keep_arc = ok[pair_of_arc]
    return src[keep_arc].astype(np.int32), dst[keep_arc].astype(np.int32)


def chung_lu(n: int, m_base: int, gamma: float, wcap: float, recip: float, cap: int, seed) -> Graph:
    """Directed Chung-Lu graph with power-law in/out weights.

    1. weights w_i ~ (i+1)^(-1/(gamma-1)), scaled to sum m_base and clipped at ``wcap``;
       in- and out-weights use independent seeded permutations of the same sequence;
    2. ``m_base`` arcs with src drawn ~ w_out and dst ~ w_in;
    3. the reverse of a seeded fraction ``recip`` of those arcs is added;
    4. self-loops and duplicates are dropped and the keyed cap is applied.
    """
    rng = _rng(seed)
    i = np.arange(n, dtype=np.float64)
    w = (i + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= m_base / w.sum()
    w = np.minimum(w, wcap)
    w_out = w[rng.permutation(n)]
    w_in = w[rng.permutation(n)]
    c_out = np.cumsum(w_out)
    c_in = np.cumsum(w_in)
    src = np.searchsorted(c_out, rng.random(m_base) * c_out[-1], side="right")
    dst = np.searchsorted(c_in, rng.random(m_base) * c_in[-1], side="right")
    src = np.minimum(src, n - 1)
    dst = np.minimum(dst, n - 1)
    rev = rng.random(m_base) < recip
    src2 = np.concatenate([src, dst[rev]])
    dst2 = np.concatenate([dst, src[rev]])
    s, d = keyed_cap(n, src2, dst2, cap, rng.integers(0, 2**63 - 1))
    return Graph(n, s, d, f"chung_lu({n},{m_base},{gamma})")


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, cap: int, seed) -> Graph:
    """R-MAT: every arc picks one of four quadrants per level with probabilities (a, b, c, d)."""
    rng = _rng(seed)
    n = 1 << scale
    m = edge_factor * n
    src = np.zeros(m, np.int64)
    dst = np.zeros(m, np.int64)
    ab = a + b
    abc = a + b + c
    chunk = 1 << 22
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        s = np.zeros(hi - lo, np.int64)
        t = np.zeros(hi - lo, np.int64)
        for _ in range(scale):
            u = rng.random(hi - lo)
            sbit = (u >= ab).astype(np.int64)                     # quadrants c, d: lower half
            tbit = ((u >= a) & (u < ab)) | (u >= abc)             # quadrants b, d: right half
            s = (s << 1) | sbit
            t = (t << 1) | tbit.astype(np.int64)
        src[lo:hi] = s
        dst[lo:hi] = t
    s, d = keyed_cap(n, src, dst, cap, rng.integers(0, 2**63 - 1))
    return Graph(n, s, d, f"rmat({scale},{edge_factor})")


def er_batch(count: int, n_lo: int, n_hi: int, mu_lo: float, mu_hi: float, seed: int) -> list[Graph]:
    """``count`` directed G(n,p) graphs; graph i uses seed (seed, i), n ~ U{n_lo..n_hi},
    mean out-degree mu ~ U[mu_lo, mu_hi] and p = mu / (n - 1)."""
    out = []
    for gi in range(count):
        rng = _rng((seed, gi))
        n = int(rng.integers(n_lo, n_hi + 1))
        mu = float(rng.uniform(mu_lo, mu_hi))
        g = er_directed(n, mu / (n - 1), (seed, gi, 1))
        g.name = f"batch[{gi}]"
        out.append(g)
    return out


def serve_pool(count: int, log_lo: float, log_hi: float, mu_lo: float, mu_hi: float, seed: int,
               gamma: float = 2.1, cap: int = 2000) -> list[Graph]:
    """A pool of graphs: even slots ER, odd slots Chung-Lu; n = round(10^U(log_lo, log_hi)),
    mean out-degree mu ~ U[mu_lo, mu_hi]."""
    out = []
    for gi in range(count):
        rng = _rng((seed, gi))
        n = int(round(10 ** rng.uniform(log_lo, log_hi)))
        mu = float(rng.uniform(mu_lo, mu_hi))
        if gi % 2 == 0:
            g = er_directed(n, mu / max(n - 1, 1), (seed, gi, 1))
        else:
            g = chung_lu(n, max(1, int(round(mu * n / 1.2))), gamma, cap / 2, 0.2, cap, (seed, gi, 2))
        g.name = f"pool[{gi}]"
        out.append(g)
    return out


def config_graph(name: str) -> Graph:
    """The named workloads.

    * ``er1000``   directed G(1000, 0.005), seed 1 (the small exact case);
    * ``chunglu``  Chung-Lu, n = 1e6, 8.4e6 base arcs, gamma 2.1, weights clipped at 1000,
                   20% reciprocated, undirected degree capped at 2000, seed 2 (~10M arcs);
    * ``rmat22``   R-MAT scale 22, edge factor 8, (0.57, 0.19, 0.19, 0.05), cap 1500, seed 4.
    """
    if name == "er1000":
        return er_directed(1000, 0.005, 1)
    if name == "chunglu":
        return chung_lu(1_000_000, 8_400_000, 2.1, 1000.0, 0.2, 2000, 2)
    if name == "rmat22":
        return rmat(22, 8, 0.57, 0.19, 0.19, 1500, 4)
    if name.startswith("chunglu_"):
        # scaled-down Chung-Lu of the same recipe, chunglu_<n>: mean degree as above,
        # weight clip and degree cap shrunk with sqrt(n / 1e6) so the hubs stay sparse
        n = int(name.split("_")[1])
        wcap = max(8.0, 1000.0 * (n / 1e6) ** 0.5)
        return chung_lu(n, int(8.4 * n), 2.1, wcap, 0.2, int(2 * wcap), 2)
    raise KeyError(name)


def special_graph(name: str, n: int) -> Graph:
    """Small graphs whose motif counts have closed forms (cliques, DAGs, cycles, stars)."""
    idx = np.arange(n)
    if name == "complete":          # every ordered pair is an arc (complete bidirected graph)
        s, d = np.nonzero(~np.eye(n, dtype=bool))
    elif name == "tournament":      # transitive tournament i -> j for i < j (a regular DAG)
        s, d = np.nonzero(np.triu(np.ones((n, n), bool), 1))
    elif name == "cycle":           # directed cycle i -> i+1 mod n
        s, d = idx, (idx + 1) % n
    elif name == "outstar":         # hub 0 -> every other vertex
        s, d = np.zeros(n - 1, np.int64), idx[1:]
    elif name == "instar":          # every other vertex -> hub 0
        s, d = idx[1:], np.zeros(n - 1, np.int64)
    elif name == "path":            # directed path i -> i+1
        s, d = idx[:-1], idx[1:]
    elif name == "empty":
        s, d = np.zeros(0, np.int64), np.zeros(0, np.int64)
    else:
        raise KeyError(name)
    return Graph(n, np.asarray(s, np.int32), np.asarray(d, np.int32), f"{name}({n})")


def describe(g: Graph) -> dict:
    return {"name": g.name, "n": g.n, "arcs": g.m, "sha256": digest(g)}
