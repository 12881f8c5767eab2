"""Writes the stored oracle rows used by the full-size parity tests.

For a named full-size workload (``chunglu``: k = 3 and 4; ``rmat22``: k = 4) this picks
the 16 vertices of largest undirected degree (ties by id) and 48 seeded random
non-isolated vertices, and computes their per-vertex rows with the oracle's per-vertex
mode (every connected k-set containing the vertex, enumerated once).  Only ``oracle/``
and the seeded generators are called.  The output, ``fullsize_<name>.txt``, starts with
the SHA-256 of the generated input and lists the non-zero entries as
``vertex k class count``; the test refuses a file whose digest differs from the input
it generates.

Usage: python tests/golden/make_fullsize_rows.py chunglu [threads]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

KS = {"chunglu": (3, 4), "rmat22": (4,)}
N_TOP, N_RANDOM, SEED = 16, 48, 2201


def undirected_degree(g):
    s, d = g.src.astype(np.int64), g.dst.astype(np.int64)
    keep = s != d
    lo, hi = np.minimum(s[keep], d[keep]), np.maximum(s[keep], d[keep])
    u = np.unique(lo * g.n + hi)
    return np.bincount(np.concatenate([u // g.n, u % g.n]), minlength=g.n)


def pick_rows(g):
    deg = undirected_degree(g)
    order = np.lexsort((np.arange(g.n), -deg))
    top = [int(x) for x in order[:N_TOP]]
    rng = np.random.default_rng(SEED)
    cand = np.setdiff1d(np.flatnonzero(deg > 0), np.array(top))
    rnd = [int(x) for x in rng.choice(cand, size=N_RANDOM, replace=False)]
    return top + rnd, deg


def main():
    name = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else oracle.default_threads()
    g = gg.config_graph(name)
    rows, deg = pick_rows(g)
    path = os.path.join(HERE, f"fullsize_{name}.txt")
    tmp = path + ".partial"
    with open(tmp, "w") as f:
        f.write(f"# oracle per-vertex rows of the {name} workload (tests/golden/make_fullsize_rows.py)\n")
        f.write(f"sha256 {gg.digest(g)}\n")
        f.write("rows " + " ".join(str(v) for v in rows) + "\n")
        for k in KS[name]:
            for v in rows:
                t0 = time.time()
                out = oracle.count_rows(g.n, g.src, g.dst, k, np.array([v], np.int32), threads=threads)[0]
                for c in np.flatnonzero(out):
                    f.write(f"{v} {k} {int(c)} {int(out[c])}\n")
                f.flush()
                print(f"{name} k={k} vertex {v} (degree {deg[v]}): {int(out.sum())} sets in "
                      f"{time.time() - t0:.1f} s", flush=True)
    os.replace(tmp, path)


if __name__ == "__main__":
    main()
