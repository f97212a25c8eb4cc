"""Writes <config>_R_sample.npz for the full-size parity tests: the float64
oracle's level-0 estimate (Alg. 1) on the netlist200k and large2m inputs,
start blocks of the counter generator (seed 7, levels 0, rounded to float32
as the library receives them).  Stored: Q_H of every pool column, and R on
8192 hyperedges drawn with numpy seed 12345 (plus the indices).  Calls only
the oracle and the seeded input generators.

    python tests/golden/make_fullsize_samples.py [netlist200k] [large2m]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import resistance as orr  # noqa: E402
from synth import get_config, make_hypergraph, start_block  # noqa: E402

NSAMPLE = 8192


def main(names):
    for name in names:
        cfg = get_config(name)
        h = make_hypergraph(name)
        k, b = cfg["k"], cfg["b"]
        Xs = start_block(7, 0, 0, h.n + h.m, b).astype(np.float32).astype(np.float64)
        Xc = start_block(7, 0, 1, h.n, b).astype(np.float32).astype(np.float64)
        t = time.time()
        R, qh = lean_resistance(h, Xs, Xc, k)
        idx = np.sort(np.random.default_rng(12345).choice(h.m, size=NSAMPLE, replace=False))
        np.savez(os.path.join(HERE, f"{name}_R_sample.npz"), idx=idx.astype(np.int64),
                 R=R[idx], qh=qh, Rmax=np.float64(R.max()), Rnorm=np.float64(np.linalg.norm(R)))
        print(f"{name}: {time.time() - t:.0f} s, max R {R.max():.4e}", flush=True)


def lean_resistance(h, Xs, Xc, k, tau=1e-3):
    """orr.resistance with the per-expansion blocks released as soon as
    their pool columns are taken, so that the 2M-node case fits in host
    memory: orr.unified_pool(keep_blocks=False), then the ratios."""
    pool = orr.unified_pool(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k, tau, keep_blocks=False)
    return orr.resistance_from_pool(h.eptr, h.pins, h.w, pool.chi)


if __name__ == "__main__":
    main(sys.argv[1:] or ["netlist200k", "large2m"])
