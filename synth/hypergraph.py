"""Seeded synthetic hypergraphs shaped like VLSI netlists.

The paper evaluates on ISPD98 and Titan23 netlists (Section IV, Tables III and
IV give their node and net counts).  Those files are not available here, so
these seeded hypergraphs stand in for them.  The recipe:

* sizes: |e| = s with probability proportional to s**-alpha on the integers
  [lo, hi] (a truncated power law);
* pins: each hyperedge gets an anchor a ~ U[0, n).  The number of local pins
  is L ~ Binomial(|e|, p_loc), capped at the window size; the local pins are a
  uniform L-subset of the window [a - win/2, a + win/2) (mod n), and the other
  |e| - L pins are a uniform subset of the remaining nodes.  p_loc = 0 gives
  pins drawn uniformly without replacement;
* hyperedges are emitted in ascending anchor order (netlist-like id locality)
  unless ``shuffle_edges`` is set;
* pins are stored ascending within each hyperedge, so they are distinct;
* weights: all 1.0, or lognormal(0, sigma) = exp(sigma * N(0, 1)), float32.

Storage is CSR over hyperedges: ``eptr[m+1]`` (int64 here; the library takes
int32) and ``pins[eptr[m]]`` (int32).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Hypergraph:
    n: int
    m: int
    eptr: np.ndarray   # int64 [m+1]
    pins: np.ndarray   # int32 [nnz], ascending within each hyperedge
    w: np.ndarray      # float32 [m], > 0

    @property
    def nnz(self) -> int:
        return int(self.eptr[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.eptr)

    def edge_ids(self) -> np.ndarray:
        return np.repeat(np.arange(self.m, dtype=np.int64), self.sizes())


def size_law(lo: int, hi: int, alpha: float):
    s = np.arange(lo, hi + 1, dtype=np.int64)
    p = s.astype(np.float64) ** (-alpha)
    return s, p / p.sum()


def _segment_has_dup(keys_sorted: np.ndarray) -> np.ndarray:
    dup = np.zeros(keys_sorted.shape[0], dtype=bool)
    dup[1:] = keys_sorted[1:] == keys_sorted[:-1]
    return dup


def generate(n: int, m: int, lo: int = 2, hi: int = 20, alpha: float = 2.5,
             p_loc: float = 0.0, win: int = 1000, weights: str = "unit",
             sigma: float = 0.5, seed: int = 0, shuffle_edges: bool = False) -> Hypergraph:
    if hi > n:
        raise ValueError("largest hyperedge exceeds the node count")
    rng = np.random.Generator(np.random.PCG64(seed))
    vals, prob = size_law(lo, hi, alpha)
    sizes = rng.choice(vals, size=m, p=prob).astype(np.int64)
    anchors = rng.integers(0, n, size=m, dtype=np.int64)
    wsz = min(win, n)
    if p_loc > 0:
        nloc = np.minimum(rng.binomial(sizes, p_loc), wsz)
    else:
        nloc = np.zeros(m, dtype=np.int64)
    if not shuffle_edges:
        order = np.argsort(anchors, kind="stable")
        sizes, anchors, nloc = sizes[order], anchors[order], nloc[order]

    eptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=eptr[1:])
    nnz = int(eptr[-1])
    eid = np.repeat(np.arange(m, dtype=np.int64), sizes)
    slot = np.arange(nnz, dtype=np.int64) - eptr[eid]
    is_local = slot < nloc[eid]
    half = wsz // 2

    def draw(idx):
        out = np.empty(idx.shape[0], dtype=np.int64)
        loc = is_local[idx]
        nl = int(loc.sum())
        out[loc] = (anchors[eid[idx[loc]]] - half + rng.integers(0, wsz, size=nl)) % n
        out[~loc] = rng.integers(0, n, size=idx.shape[0] - nl)
        return out

    # Hyperedges whose local part fills a large share of the window draw it
    # as a random subset directly (rejection would stall like a coupon collector).
    big = np.nonzero(nloc > wsz // 4)[0]
    pins = draw(np.arange(nnz, dtype=np.int64))
    for e in big:
        L = int(nloc[e])
        offs = rng.choice(wsz, size=L, replace=False)
        pins[eptr[e]:eptr[e] + L] = (anchors[e] - half + offs) % n

    # Reject duplicates: redraw the later copy until every hyperedge is a set.
    active = np.arange(m, dtype=np.int64)
    for _ in range(10000):
        if active.size == 0:
            break
        sel_sizes = sizes[active]
        idx = np.repeat(eptr[active], sel_sizes) + (
            np.arange(int(sel_sizes.sum()), dtype=np.int64)
            - np.repeat(np.cumsum(sel_sizes) - sel_sizes, sel_sizes))
        key = eid[idx] * n + pins[idx]
        o = np.argsort(key, kind="stable")
        dup_sorted = _segment_has_dup(key[o])
        if not dup_sorted.any():
            break
        redo = idx[o[dup_sorted]]
        # never redraw a directly sampled window subset
        pins[redo] = draw(redo)
        active = np.unique(eid[redo])
    else:  # pragma: no cover
        raise RuntimeError("duplicate rejection did not converge")

    # ascending pins within each hyperedge
    key = eid * n + pins
    pins = (np.sort(key) - eid * n).astype(np.int32)

    if weights == "unit":
        w = np.ones(m, dtype=np.float32)
    elif weights == "lognormal":
        w = np.exp(sigma * rng.standard_normal(m)).astype(np.float32)
    else:
        raise ValueError(f"unknown weight law {weights!r}")
    return Hypergraph(n=n, m=m, eptr=eptr, pins=pins, w=w)
