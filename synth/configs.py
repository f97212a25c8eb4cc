"""The benchmark and parity workloads, by name.

Each workload fixes the hypergraph recipe (see ``synth.hypergraph``) and the
method's parameters: k Krylov steps per expansion, b start vectors per
expansion (pool width K = 2*b*k), coarsening levels and the merge percentile.
"""
from __future__ import annotations

import numpy as np

from .hypergraph import Hypergraph, generate

HG_SEED_BASE = 20251106
START_SEED = 7

CONFIGS = {
    # 2,000 nodes / 2,000 nets, sizes ~ s^-2.5 on [2,20], uniform pins, unit w
    "tiny2k": dict(index=0, n=2000, m=2000, lo=2, hi=20, alpha=2.5, p_loc=0.0,
                   weights="unit", k=10, b=1, levels=1, percentile=0.5,
                   local_clustering=True),
    # 50-node variant of the tiny recipe, small enough for pseudo-inverses
    "pinv50": dict(index=0, n=50, m=50, lo=2, hi=20, alpha=2.5, p_loc=0.0,
                   weights="unit", k=10, b=1, levels=1, percentile=0.5,
                   local_clustering=True),
    # IBM18-sized netlist: 200k nodes, 210k nets, sizes on [2,2000] (mean 3.6)
    "netlist200k": dict(index=1, n=200_000, m=210_000, lo=2, hi=2000, alpha=2.7828,
                        p_loc=0.7, weights="unit", k=20, b=4, levels=3,
                        percentile=0.5, local_clustering=True),
    # headline: 2M nodes, 2.2M nets, lognormal(0, 0.5) weights
    "large2m": dict(index=2, n=2_000_000, m=2_200_000, lo=2, hi=2000, alpha=2.7828,
                    p_loc=0.7, weights="lognormal", k=30, b=8, levels=3,
                    percentile=0.5, local_clustering=True),
    # gradient workload: the 200k generator with lognormal weights, level 0 only
    "grad200k": dict(index=3, n=200_000, m=210_000, lo=2, hi=2000, alpha=2.7828,
                     p_loc=0.7, weights="lognormal", k=20, b=4, levels=1,
                     percentile=0.5, local_clustering=False),
    # precision workload: 10M nodes, 11M nets, BF16 pool
    "bf16_10m": dict(index=4, n=10_000_000, m=11_000_000, lo=2, hi=2000, alpha=2.7828,
                     p_loc=0.7, weights="lognormal", k=30, b=8, levels=3,
                     percentile=0.5, local_clustering=True),
}


def get_config(name: str) -> dict:
    return dict(CONFIGS[name])


def make_hypergraph(name: str, seed: int | None = None, **override) -> Hypergraph:
    c = get_config(name)
    c.update(override)
    if seed is None:
        seed = HG_SEED_BASE + c["index"]
    return generate(c["n"], c["m"], lo=c["lo"], hi=c["hi"], alpha=c["alpha"],
                    p_loc=c["p_loc"], weights=c["weights"], seed=seed)


def graph_2uniform(n: int = 50, m: int = 120, seed: int = HG_SEED_BASE) -> Hypergraph:
    """A random simple graph as a 2-uniform hypergraph (every |e| = 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = set()
    # a spanning path keeps it connected
    perm = rng.permutation(n)
    for i in range(n - 1):
        a, b = sorted((int(perm[i]), int(perm[i + 1])))
        edges.add((a, b))
    while len(edges) < m:
        a, b = rng.integers(0, n, size=2)
        if a != b:
            edges.add((int(min(a, b)), int(max(a, b))))
    edges = sorted(edges)
    pins = np.array(edges, dtype=np.int32).reshape(-1)
    eptr = np.arange(0, 2 * len(edges) + 1, 2, dtype=np.int64)
    w = np.exp(0.5 * rng.standard_normal(len(edges))).astype(np.float32)
    return Hypergraph(n=n, m=len(edges), eptr=eptr, pins=pins, w=w)
