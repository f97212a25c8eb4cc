"""Cluster quality: hypergraph conductance and its average, in plain NumPy.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Passages followed (HyperEF 2.0):
* Section II-A "Hypergraph conductance", Eq. (3): a node's degree is the sum
  of the weights of its hyperedges, a set's volume the sum of its nodes'
  degrees, and the conductance of S is the cut between S and its complement
  divided by the smaller of the two volumes;
* Section IV, Eq. (18): the average conductance of a clustering is the mean
  of its clusters' conductances.

Readings of silent points:
* the cut counts each hyperedge with pins on both sides once, with its
  weight (the hyperedge count for unit weights);
* a cluster with a zero cut has conductance 0, including the 0/0 cases (a
  cluster of nodes without hyperedges, or a single cluster holding every
  node);
* sums run in float64.
"""
from __future__ import annotations

import numpy as np


def degrees(n, eptr, pins, w):
    """d_v = sum of w(e) over the hyperedges e that hold v (Section II-A)."""
    m = len(eptr) - 1
    d = np.zeros(n, dtype=np.float64)
    for e in range(m):
        for v in pins[eptr[e]:eptr[e + 1]]:
            d[v] += float(w[e])
    return d


def cluster_conductance(n, eptr, pins, w, label, n_clusters):
    """Per-cluster (cut, vol, phi) of Eq. (3) for the partition label[n] in
    [0, n_clusters).  w = None means unit weights."""
    m = len(eptr) - 1
    w = np.ones(m) if w is None else np.asarray(w, dtype=np.float64)
    label = np.asarray(label)
    cut = np.zeros(n_clusters, dtype=np.float64)
    for e in range(m):
        touched = set(int(label[v]) for v in pins[eptr[e]:eptr[e + 1]])
        if len(touched) > 1:
            for c in touched:
                cut[c] += w[e]
    d = degrees(n, eptr, pins, w)
    vol = np.zeros(n_clusters, dtype=np.float64)
    for v in range(n):
        vol[label[v]] += d[v]
    total = float(d.sum())
    phi = np.zeros(n_clusters, dtype=np.float64)
    for c in range(n_clusters):
        if cut[c] != 0.0:
            phi[c] = cut[c] / min(vol[c], total - vol[c])
    return cut, vol, phi


def average_conductance(phi):
    """Phi_avg of Eq. (18): the mean of the clusters' conductances."""
    phi = np.asarray(phi, dtype=np.float64)
    return float(phi.sum() / len(phi)) if len(phi) else 0.0


def one_cluster(eptr, pins, w, label, c):
    """(cut, vol) of the single cluster c, for sampled checks on large
    inputs: a hyperedge with k of its |e| pins in c adds w(e) to the volume
    k times and to the cut once when 0 < k < |e| (the same quantities as
    cluster_conductance, one cluster at a time, vectorised)."""
    eptr = np.asarray(eptr)
    m = len(eptr) - 1
    w = np.ones(m) if w is None else np.asarray(w, dtype=np.float64)
    sizes = np.diff(eptr)
    inside = np.add.reduceat((np.asarray(label)[pins] == c).astype(np.int64), eptr[:-1]) \
        if m else np.zeros(0, np.int64)
    touched = inside > 0
    split = touched & (inside < sizes)
    return float(w[split].sum()), float((w * inside).sum())
