"""Alg. 2's level loop: Alg. 1 on the current hypergraph, then one level of
contraction, local clustering and rebuild, repeated for a fixed number of
levels.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Start blocks are inputs: ``start(level, expansion, rows, b)`` returns the
rows x b block of that level (expansion 0 = star over n+m rows, 1 = clique
over n rows).  ``levels`` runs that many levels; with ``target_nr`` > 0 it
is a cap and the loop stops earlier, at the node-reduction ratio of
Section IV (NR = 60 % is a 2.5x reduction): before a level once the node
count has reached (1 - NR) n_0, or after a level that merged nothing.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import clustering, resistance


@dataclass
class CoarsenResult:
    cluster: np.ndarray      # original node -> final label
    n_clusters: int
    R0: np.ndarray           # level-0 resistances (Alg. 1 output)
    eta: np.ndarray          # eta of every final cluster
    levels: list             # per-level (n, m, nnz, LevelResult)


def coarsen(n, m, eptr, pins, w, k, b, levels, start, percentile=0.5,
            local_clustering=True, tau=1e-3, target_nr=0.0, **kw) -> CoarsenResult:
    eptr = np.asarray(eptr, dtype=np.int64)
    pins = np.asarray(pins, dtype=np.int64)
    w = np.asarray(w, dtype=np.float32)
    mapping = np.arange(n, dtype=np.int64)
    eta = np.zeros(n, dtype=np.float32)
    R0 = None
    info = []
    n0 = n
    goal = (1.0 - float(np.float32(target_nr))) * float(n0)
    for level in range(levels):
        if m == 0:
            break
        if target_nr > 0 and n <= goal:
            break
        est = resistance.resistance(n, m, eptr, pins, w, start(level, 0, n + m, b),
                                    start(level, 1, n, b), k, tau, **kw)
        if R0 is None:
            R0 = est.R
        lev = clustering.cluster_level(n, m, eptr, pins, est.R, eta, est.pool.chi,
                                       est.qh, percentile, local_clustering)
        info.append((n, m, int(eptr[-1]), lev))
        mapping = lev.label[mapping].astype(np.int64)
        m, eptr, pins, w, _ = clustering.rebuild(m, eptr, pins, w, lev.label)
        pins = pins.astype(np.int64)
        stalled = lev.n_clusters == n
        n, eta = lev.n_clusters, lev.eta
        if target_nr > 0 and stalled:
            break
    if R0 is None:
        R0 = np.zeros(0)
    return CoarsenResult(cluster=mapping.astype(np.int32), n_clusters=int(n), R0=R0,
                         eta=eta, levels=info)
