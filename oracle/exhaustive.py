"""Plain-definition oracle over all k-subsets, pure Python (tiny graphs only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For every k-subset S of the vertices (Sec. 4.1: a k-motif is a set of k vertices
connected in the undirected graph underneath G):
  * skip S unless it is connected in G_U;
  * read its induced adjacency matrix in any vertex order as the motif index
    (rows in order, diagonal dropped, first entry most significant; Sec. 4.1, Fig. 1);
  * map the index to the minimal index over all k! relabellings (Fig. 1, Sec. 4.2);
  * add one to that class's counter of every vertex of S (Sec. 4.2).
Class ids are the minimal indices of connected motifs in ascending order.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np


def motif_index(A) -> int:
    """Index of a k x k 0/1 matrix: entries row by row, diagonal skipped, first = MSB."""
    k = len(A)
    bits = [A[i][j] for i in range(k) for j in range(k) if i != j]
    v = 0
    for b in bits:
        v = (v << 1) | (1 if b else 0)
    return v


def matrix_of(k: int, code: int):
    pos = [(i, j) for i in range(k) for j in range(k) if i != j]
    A = [[0] * k for _ in range(k)]
    L = len(pos)
    for t, (i, j) in enumerate(pos):
        A[i][j] = (code >> (L - 1 - t)) & 1
    return A


def minimal_index(k: int, code: int) -> int:
    A = matrix_of(k, code)
    best = None
    for p in itertools.permutations(range(k)):
        B = [[A[p[i]][p[j]] for j in range(k)] for i in range(k)]
        c = motif_index(B)
        best = c if best is None or c < best else best
    return best


def weakly_connected(A) -> bool:
    k = len(A)
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for y in range(k):
            if y not in seen and (A[x][y] or A[y][x]):
                seen.add(y)
                stack.append(y)
    return len(seen) == k


def classes(k: int):
    """(minimal index of every code, sorted list of connected class codes)."""
    n_codes = 1 << (k * (k - 1))
    mins = [minimal_index(k, c) for c in range(n_codes)]
    conn = sorted({mins[c] for c in range(n_codes) if weakly_connected(matrix_of(k, c))})
    return mins, conn


@functools.lru_cache(maxsize=None)
def _minimal_index_cached(k: int, code: int) -> int:
    return minimal_index(k, code)


def count_by_code(n: int, src, dst, k: int):
    """Brute force keyed by the minimal index itself rather than by a class id, so that it
    needs no table of all 2^(k(k-1)) codes (k = 5 has 2^20): ({min index: uint64[n]}
    per-vertex counts, {min index: total}), over every connected k-subset."""
    arcs = set()
    for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if u != v:
            arcs.add((u, v))
    und = [set() for _ in range(n)]
    for u, v in arcs:
        und[u].add(v)
        und[v].add(u)
    rows, tot = {}, {}
    for S in itertools.combinations(range(n), k):
        seen, stack, members = {S[0]}, [S[0]], set(S)
        while stack:
            x = stack.pop()
            for y in und[x]:
                if y in members and y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) != k:
            continue
        A = [[1 if (i != j and (S[i], S[j]) in arcs) else 0 for j in range(k)] for i in range(k)]
        m = _minimal_index_cached(k, motif_index(A))
        if m not in rows:
            rows[m] = np.zeros(n, np.uint64)
            tot[m] = 0
        tot[m] += 1
        for v in S:
            rows[m][v] += 1
    return rows, tot


def count(n: int, src, dst, k: int):
    """uint64[n][C] per-vertex counts and uint64[C] totals, by brute force."""
    arcs = set()
    for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if u != v:
            arcs.add((u, v))
    und = [set() for _ in range(n)]
    for u, v in arcs:
        und[u].add(v)
        und[v].add(u)
    mins, conn = classes(k)
    cid = {c: i for i, c in enumerate(conn)}
    out = np.zeros((n, len(conn)), np.uint64)
    tot = np.zeros(len(conn), np.uint64)
    for S in itertools.combinations(range(n), k):
        # connectivity in G_U
        seen = {S[0]}
        stack = [S[0]]
        members = set(S)
        while stack:
            x = stack.pop()
            for y in und[x]:
                if y in members and y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) != k:
            continue
        A = [[1 if (i != j and (S[i], S[j]) in arcs) else 0 for j in range(k)] for i in range(k)]
        c = cid[mins[motif_index(A)]]
        tot[c] += 1
        for v in S:
            out[v, c] += 1
    return out, tot


# ------------------------------------------------------------------ undirected motifs

UNDIRECTED_NAMES = {
    3: ["path", "triangle"],
    4: ["path", "star", "cycle", "paw", "diamond", "clique"],
}


def undirected_name(k: int, edges) -> str:
    """Name of a connected undirected graph on k vertices from its edge count and
    degree sequence (enough to tell all 2 + 6 of them apart)."""
    deg = [0] * k
    for i, j in edges:
        deg[i] += 1
        deg[j] += 1
    m, top = len(edges), max(deg)
    if k == 3:
        return "triangle" if m == 3 else "path"
    if m == 3:
        return "star" if top == 3 else "path"
    if m == 4:
        return "paw" if top == 3 else "cycle"
    return "diamond" if m == 5 else "clique"


def count_undirected(n: int, src, dst, k: int):
    """{name: uint64[n]} per-vertex counts of the connected induced subgraphs of G_U,
    by brute force over all k-subsets (arc directions ignored)."""
    und = [set() for _ in range(n)]
    for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if u != v:
            und[u].add(v)
            und[v].add(u)
    out = {name: np.zeros(n, np.uint64) for name in UNDIRECTED_NAMES[k]}
    for S in itertools.combinations(range(n), k):
        edges = [(i, j) for i in range(k) for j in range(i + 1, k) if S[j] in und[S[i]]]
        seen, stack = {0}, [0]
        while stack:
            x = stack.pop()
            for i, j in edges:
                y = j if i == x else (i if j == x else None)
                if y is not None and y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) != k:
            continue
        name = undirected_name(k, edges)
        for v in S:
            out[name][v] += 1
    return out


# ------------------------------------------------------------------ per-edge counts

def count_edges(n: int, src, dst, k: int):
    """(pairs, uint64[P][C]): pairs = sorted list of the G_U pairs (lo < hi); row p counts,
    per class, the connected k-sets containing both endpoints.  Brute force."""
    arcs = set()
    for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if u != v:
            arcs.add((u, v))
    pairs = sorted({(min(u, v), max(u, v)) for u, v in arcs})
    pid = {pr: i for i, pr in enumerate(pairs)}
    und = [set() for _ in range(n)]
    for u, v in arcs:
        und[u].add(v)
        und[v].add(u)
    mins, conn = classes(k)
    cid = {c: i for i, c in enumerate(conn)}
    out = np.zeros((len(pairs), len(conn)), np.uint64)
    for S in itertools.combinations(range(n), k):
        seen, stack, members = {S[0]}, [S[0]], set(S)
        while stack:
            x = stack.pop()
            for y in und[x]:
                if y in members and y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) != k:
            continue
        A = [[1 if (i != j and (S[i], S[j]) in arcs) else 0 for j in range(k)] for i in range(k)]
        c = cid[mins[motif_index(A)]]
        for i in range(k):
            for j in range(i + 1, k):
                if S[j] in und[S[i]]:
                    out[pid[(min(S[i], S[j]), max(S[i], S[j]))], c] += 1
    return pairs, out
