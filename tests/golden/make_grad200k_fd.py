"""Writes grad200k_fd.npz: central finite differences of the float64 oracle's
L(w) = sum_e c_e R_e(w) at the full gradient workload (200k nodes, 210k
hyperedges, lognormal weights, k = 20, b = 4; the start blocks and c of
make_grad200k.py) on 64 hyperedge weights drawn with numpy seed 13, step
h = 1e-3 w_j.  Stored per index: the difference quotient and how many of
the forward's maxima take another branch at w_j +- h (the ratio column of
Eq. (14) per hyperedge; the largest and smallest pin per hyperedge and
column).  At this size some near-tie somewhere always switches; the quotient
stays a derivative up to the jumps of those few terms.  Calls only the oracle
and the seeded input generators.

    python tests/golden/make_grad200k_fd.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import resistance as orr  # noqa: E402
from synth import get_config, make_hypergraph, start_block  # noqa: E402

NIDX = 64
REL_STEP = 1e-3


def main():
    cfg = get_config("grad200k")
    h = make_hypergraph("grad200k")
    k, b = cfg["k"], cfg["b"]
    Xs = start_block(7, 0, 0, h.n + h.m, b).astype(np.float32).astype(np.float64)
    Xc = start_block(7, 0, 1, h.n, b).astype(np.float32).astype(np.float64)
    coef = np.random.default_rng(7).standard_normal(h.m)
    idx = np.sort(np.random.default_rng(13).choice(h.m, size=NIDX, replace=False))
    w0 = h.w.astype(np.float64)
    eptr = np.asarray(h.eptr, dtype=np.int64)

    P = eptr[-1]
    eid = np.repeat(np.arange(h.m), np.diff(eptr))
    pos = np.arange(P)[:, None]

    def forward(w):
        est = orr.resistance(h.n, h.m, h.eptr, h.pins, w, Xs, Xc, k)
        G = est.pool.chi[h.pins]
        hi = np.maximum.reduceat(G, eptr[:-1], axis=0)
        lo = np.minimum.reduceat(G, eptr[:-1], axis=0)
        s = (hi - lo) ** 2
        col = (s / est.qh[None, :]).argmax(1)
        # first CSR position of the largest and smallest pin per hyperedge
        # and column
        ahi = np.minimum.reduceat(np.where(G == hi[eid], pos, P), eptr[:-1], axis=0)
        alo = np.minimum.reduceat(np.where(G == lo[eid], pos, P), eptr[:-1], axis=0)
        return float(coef @ est.R), col, ahi, alo

    t0 = time.time()
    _, c0, h0, l0 = forward(w0)
    print(f"base forward {time.time() - t0:.0f} s", flush=True)
    fd = np.zeros(NIDX)
    ncol = np.zeros(NIDX, dtype=np.int64)   # hyperedges whose ratio column switches
    npin = np.zeros(NIDX, dtype=np.int64)   # (hyperedge, column) extreme pins switching
    for t, i in enumerate(idx):
        step = REL_STEP * w0[i]
        wp, wm = w0.copy(), w0.copy()
        wp[i] += step
        wm[i] -= step
        Lp, cp, hp, lp = forward(wp)
        Lm, cm, hm, lm = forward(wm)
        fd[t] = (Lp - Lm) / (2 * step)
        ncol[t] = int(((cp != c0) | (cm != c0)).sum())
        npin[t] = int(((hp != h0) | (hm != h0) | (lp != l0) | (lm != l0)).sum())
        print(f"{t + 1}/{NIDX} index {i}: fd {fd[t]:.6e} column switches {ncol[t]} "
              f"pin switches {npin[t]} ({time.time() - t0:.0f} s)", flush=True)
    np.savez(os.path.join(HERE, "grad200k_fd.npz"), idx=idx.astype(np.int64), fd=fd,
             column_switches=ncol, pin_switches=npin, rel_step=np.float64(REL_STEP))


if __name__ == "__main__":
    main()
