"""Alg. 2 (resistance-based hypergraph local clustering) in plain NumPy.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Passages followed (HyperEF 2.0):
* Section III-A "Multilevel Effective Resistance Clustering": hyperedges with
  R_e < delta are contracted, each new supernode weighs the resistance of the
  hyperedge that formed it, and Eq. (15) adds the pins' weights eta(v) to R_e
  at the next level (eta = 0 on the original hypergraph);
* Alg. 1 and Alg. 2: contraction starts from the lowest resistances;
* Section III-B: isolated nodes (those left ungrouped by the contraction)
  look at the clusters met through their hyperedges (Eq. (16)), measure the
  distance with the numerator of Eq. (13) against the mean chi-vector of each
  cluster, and merge with the nearest one; the merged cluster's resistance is
  updated in the manner of Eq. (15);
* Alg. 2, from the resistance update to the local clustering.

Readings of silent points (all deterministic, so that a parallel
implementation can reproduce them bit for bit):
* Eq. (15) sums eta over the pins in CSR order in float64, adds R_e, and
  rounds to float32;
* delta is the nearest-rank lower percentile: sort(R_upd)[ceil(pi*m) - 1];
  contraction needs R_upd < delta strictly;
* contraction is the sequential greedy over hyperedges in ascending
  (R_upd, e) order that contracts e when none of its pins is taken yet;
* the distance of Eq. (13)'s numerator is taken in resistance units,
  d(p, C) = max_i (chi_p^(i) - c_C^(i))^2 / Q_H(chi^(i)), over columns with
  Q_H > 0, in float64 with every operation rounded separately;
* a centroid is the float64 sum of its members' rows in ascending node order
  divided by the member count;
* every isolated node with at least one hyperedge picks the candidate with
  the smallest distance, ties to the smallest label; all picks are applied at
  once (union-find over the pairs {p, best(p)});
* a merged cluster's eta is the float64 sum of its parts' eta in ascending
  label order followed by the distances of its distinct attach pairs in
  ascending (min, max) order, rounded to float32;
* labels are ranks of each cluster's smallest node id;
* the coarse hypergraph maps pins to labels, removes repeated labels, drops
  hyperedges left with fewer than 2 pins, and keeps weights and edge order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _positions(eptr: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    sizes = np.diff(eptr)
    eid = np.repeat(np.arange(sizes.shape[0], dtype=np.int64), sizes)
    pos = np.arange(eptr[-1], dtype=np.int64) - eptr[eid]
    return eid, pos


def sequential_segment_sum(eptr: np.ndarray, vals: np.ndarray, init=None) -> np.ndarray:
    """acc_e = init_e + v_0 + v_1 + ... over each segment, left to right, in
    float64 (the loop runs over the position inside the segment, so each
    segment is summed strictly in order)."""
    eptr = np.asarray(eptr, dtype=np.int64)
    m = eptr.shape[0] - 1
    sizes = np.diff(eptr)
    acc = np.zeros((m,) + vals.shape[1:]) if init is None else np.array(init, dtype=np.float64)
    vals = np.asarray(vals, dtype=np.float64)
    for t in range(int(sizes.max()) if m else 0):
        sel = np.nonzero(sizes > t)[0]
        acc[sel] = acc[sel] + vals[eptr[sel] + t]
    return acc


def eta_update(eptr, pins, R, eta) -> np.ndarray:
    """Eq. (15): R_e <- sum_{v in e} eta(v) + R_e, rounded to float32."""
    s = sequential_segment_sum(eptr, np.asarray(eta, dtype=np.float64)[np.asarray(pins, dtype=np.int64)])
    return (s + np.asarray(R, dtype=np.float64)).astype(np.float32)


def threshold(R_upd: np.ndarray, percentile: float) -> np.float32:
    """delta = the ceil(pi*m)-th smallest R_upd."""
    m = R_upd.shape[0]
    idx = max(1, int(np.ceil(percentile * m))) - 1
    return np.sort(R_upd)[idx]


def greedy_contract(n, eptr, pins, R_upd, delta):
    """Sequential greedy in ascending (R_upd, e): contract e if R_upd < delta
    and no pin of e is taken.  Returns (owner[n] = contracting edge or -1,
    list of contracted edges in contraction order)."""
    order = np.lexsort((np.arange(R_upd.shape[0]), R_upd))
    owner = np.full(n, -1, dtype=np.int64)
    contracted = []
    for e in order:
        if not R_upd[e] < delta:
            break
        mem = pins[eptr[e]:eptr[e + 1]]
        if (owner[mem] < 0).all():
            owner[mem] = e
            contracted.append(int(e))
    return owner, contracted


@dataclass
class LevelResult:
    label: np.ndarray        # [n_l] node -> canonical label at level l+1
    n_clusters: int
    eta: np.ndarray          # [n_clusters] float32
    R_upd: np.ndarray        # [m_l] float32
    delta: float
    contracted: list
    best: dict               # isolated node -> chosen provisional label
    dist: dict               # isolated node -> its distance to best


def centroids(prov: np.ndarray, chi: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Mean chi-vector of every provisional cluster, members summed in
    ascending node order (float64).  Returns (labels, centroid rows, sizes)."""
    n = prov.shape[0]
    order = np.lexsort((np.arange(n), prov))          # by cluster, then node id
    labs, start, cnt = np.unique(prov[order], return_index=True, return_counts=True)
    eptr = np.concatenate([start, [n]]).astype(np.int64)
    sums = sequential_segment_sum(eptr, np.asarray(chi, dtype=np.float64)[order])
    return labs, sums / cnt[:, None].astype(np.float64), cnt


def distance(chi_p: np.ndarray, cent: np.ndarray, qh: np.ndarray) -> np.ndarray:
    """d(p, C) = max over usable columns of (chi_p - c_C)^2 / Q_H; 0 if none."""
    use = qh > 0
    if not use.any():
        return np.zeros(cent.shape[0])
    diff = np.asarray(chi_p, dtype=np.float64)[None, use] - cent[:, use]
    sq = diff * diff
    return (sq / qh[use][None, :]).max(axis=1)


def cluster_level(n, m, eptr, pins, R, eta, chi, qh, percentile=0.5,
                  local_clustering=True) -> LevelResult:
    """One level of Alg. 2, resistance update to local clustering, on
    H_l = (n, m, eptr, pins)."""
    eptr = np.asarray(eptr, dtype=np.int64)
    pins = np.asarray(pins, dtype=np.int64)
    eta = np.zeros(n, dtype=np.float32) if eta is None else np.asarray(eta, dtype=np.float32)
    qh = np.asarray(qh, dtype=np.float64)
    # step 4: Eq. (15)
    R_upd = eta_update(eptr, pins, R, eta)
    delta = threshold(R_upd, percentile) if m else np.float32(0)
    # step 5: contraction
    owner, contracted = greedy_contract(n, eptr, pins, R_upd, delta)
    # provisional label = smallest member node id
    prov = np.arange(n, dtype=np.int64)
    prov_eta = {}
    for e in contracted:
        mem = pins[eptr[e]:eptr[e + 1]]
        prov[mem] = mem.min()
        prov_eta[int(mem.min())] = np.float32(R_upd[e])
    is_single = owner < 0
    cl_eta = {int(v): np.float32(eta[v]) for v in np.nonzero(is_single)[0]}
    cl_eta.update(prov_eta)

    best, dist = {}, {}
    if local_clustering and n:
        labs, cent, _ = centroids(prov, chi)
        row_of = {int(l): i for i, l in enumerate(labs)}
        # CSC incidence: hyperedges of every node
        eid = np.repeat(np.arange(m, dtype=np.int64), np.diff(eptr))
        byn = np.argsort(pins, kind="stable")
        vptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(pins, minlength=n), out=vptr[1:])
        node_edges = eid[byn]
        for p in np.nonzero(is_single)[0]:
            es = node_edges[vptr[p]:vptr[p + 1]]
            if es.size == 0:
                continue
            nb = np.concatenate([pins[eptr[e]:eptr[e + 1]] for e in es])
            nb = nb[nb != p]
            cand = np.unique(prov[nb])                 # Eq. (16), as clusters
            d = distance(chi[p], cent[[row_of[int(c)] for c in cand]], qh)
            j = int(np.argmin(d))                      # first minimum = smallest label
            best[int(p)] = int(cand[j])
            dist[int(p)] = float(d[j])

    # union-find over {p, best(p)} on provisional labels
    parent = {}

    def find(x):
        while parent.get(x, x) != x:
            x = parent[x]
        return x

    for p, c in best.items():
        a, b = find(p), find(c)
        if a != b:
            parent[max(a, b)] = min(a, b)

    # final labels: component root = smallest provisional label in it
    comp = np.array([find(int(l)) for l in prov], dtype=np.int64)
    roots = np.unique(comp)
    label = np.searchsorted(roots, comp).astype(np.int32)

    # eta of every component
    members = {}
    for l in sorted(cl_eta):
        members.setdefault(find(l), []).append(l)
    pairs = {}
    for p, c in best.items():
        key = (min(p, c), max(p, c))
        pairs.setdefault(key, dist[p])
    pairs_by_root = {}
    for key in sorted(pairs):
        pairs_by_root.setdefault(find(key[0]), []).append(pairs[key])
    eta_out = np.zeros(roots.shape[0], dtype=np.float32)
    for i, r in enumerate(roots):
        acc = 0.0
        for l in members[int(r)]:
            acc += float(cl_eta[l])
        for dv in pairs_by_root.get(int(r), []):
            acc += dv
        eta_out[i] = np.float32(acc)
    return LevelResult(label=label, n_clusters=int(roots.shape[0]), eta=eta_out,
                       R_upd=R_upd, delta=float(delta), contracted=contracted,
                       best=best, dist=dist)


def rebuild(m, eptr, pins, w, label):
    """Alg. 2's coarse hypergraph over the labels (sorted unique pins,
    hyperedges with fewer than 2 labels removed, weights and order kept).
    Returns (m', eptr', pins', w', kept hyperedge ids)."""
    eptr = np.asarray(eptr, dtype=np.int64)
    new_pins, new_ptr, kept = [], [0], []
    for e in range(m):
        lab = np.unique(label[pins[eptr[e]:eptr[e + 1]]])
        if lab.size >= 2:
            new_pins.append(lab)
            new_ptr.append(new_ptr[-1] + lab.size)
            kept.append(e)
    kept = np.asarray(kept, dtype=np.int64)
    P = np.concatenate(new_pins).astype(np.int32) if new_pins else np.zeros(0, np.int32)
    return len(kept), np.asarray(new_ptr, dtype=np.int64), P, np.asarray(w)[kept], kept
