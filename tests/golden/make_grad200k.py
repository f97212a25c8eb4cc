"""Writes grad200k_dw.npz: the float64 oracle gradient of L = sum_e c_e R_e
at the full gradient workload (200k nodes, 210k hyperedges, lognormal
weights, k = 20, b = 4; start blocks of the counter generator, seed 7,
rounded to float32 as the library receives them; c ~ N(0, 1) with numpy
seed 7).  Calls only the oracle and the seeded input generators.

    python tests/golden/make_grad200k.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import gradient as ogr  # noqa: E402
from synth import get_config, make_hypergraph, start_block  # noqa: E402


def main():
    cfg = get_config("grad200k")
    h = make_hypergraph("grad200k")
    k, b = cfg["k"], cfg["b"]
    Xs = start_block(7, 0, 0, h.n + h.m, b).astype(np.float32).astype(np.float64)
    Xc = start_block(7, 0, 1, h.n, b).astype(np.float32).astype(np.float64)
    coef = np.random.default_rng(7).standard_normal(h.m)
    L, g, R = ogr.loss_and_grad(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k, coef)
    np.savez(os.path.join(HERE, "grad200k_dw.npz"), dw=g.astype(np.float32), L=np.float64(L),
             R=R.astype(np.float32))
    print(f"L = {L:.9e}, |dw| = {np.linalg.norm(g):.6e}")


if __name__ == "__main__":
    main()
