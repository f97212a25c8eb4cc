"""Resistance-based vertex-pair rating (Section III-E, Eq. (17)) in plain
Python/NumPy.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

r(p, q) = sum over the hyperedges e that hold both p and q of
w(e) / (R_e - shift): Eq. (7)'s rating with the cardinality term replaced
by the effective resistance.  Readings (stated where the library declares
the call): shift = 0 replaces the whole term |e| - 1 by R_e; shift = 1 is the
printed R_e - 1; a hyperedge whose denominator is exactly 0 adds nothing;
sums run in float64 over the hyperedges in ascending order; the best
neighbour is the one of largest rating, ties to the smallest id, -1 (rating
0) for a node without neighbours.
"""
from __future__ import annotations

import numpy as np


def node_edges(n, eptr, pins):
    """The hyperedges of every node, ascending."""
    eptr = np.asarray(eptr, dtype=np.int64)
    out = [[] for _ in range(n)]
    for e in range(len(eptr) - 1):
        for p in pins[eptr[e]:eptr[e + 1]]:
            out[int(p)].append(e)
    return out


def pair_ratings(p, edges_of_p, eptr, pins, w, R, shift=0.0):
    """{q: r(p, q)} for every q sharing a hyperedge with p."""
    sh = float(np.float32(shift))
    acc = {}
    for e in edges_of_p:
        den = float(np.float32(R[e])) - sh
        t = float(np.float32(w[e])) / den if den != 0.0 else None
        for q in pins[eptr[e]:eptr[e + 1]]:
            q = int(q)
            if q == p:
                continue
            if q not in acc:
                acc[q] = 0.0
            if t is not None:
                acc[q] = acc[q] + t
    return acc


def best_neighbours(n, m, eptr, pins, w, R, shift=0.0, nodes=None):
    """(best [n] int32, rating [n] float64) -- or for the given nodes only."""
    eptr = np.asarray(eptr, dtype=np.int64)
    pins = np.asarray(pins, dtype=np.int64)
    w = np.ones(m, np.float32) if w is None else np.asarray(w, np.float32)
    ne = node_edges(n, eptr, pins)
    sel = range(n) if nodes is None else nodes
    best = np.full(len(sel), -1, dtype=np.int32)
    val = np.zeros(len(sel))
    for i, p in enumerate(sel):
        acc = pair_ratings(int(p), ne[int(p)], eptr, pins, w, R, shift)
        if acc:
            top = max(acc.values())
            best[i] = min(q for q, v in acc.items() if v == top)
            val[i] = top
    return best, val
