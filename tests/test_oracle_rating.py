"""Pins of the oracle's Eq. (17) rating: hand-worked values, the special
case that is Eq. (7) (KaHyPar's heavy-edge rating, by brute force over the
vertex pairs of every hyperedge), and the symmetry r(p, q) = r(q, p)."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import rating as ort
from synth import generate

GOLD = os.path.join(os.path.dirname(__file__), "golden", "rating_examples.json")


def _csr(edges):
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    return eptr, np.array([p for e in edges for p in e], dtype=np.int64)


@pytest.mark.parametrize("case", json.load(open(GOLD))["cases"], ids=lambda c: f"shift{c['shift']}")
def test_hand_worked(case):
    ex = json.load(open(GOLD))
    eptr, pins = _csr(ex["edges"])
    best, val = ort.best_neighbours(ex["n"], len(ex["edges"]), eptr, pins,
                                    np.array(ex["w"], np.float32), np.array(ex["R"], np.float32),
                                    case["shift"])
    assert best.tolist() == case["best"]
    assert np.allclose(val, case["rating"], rtol=1e-15, atol=0)


def test_equation_7_special_case():
    """R_e = |e| with shift = 1 gives sum w(e) / (|e| - 1) (Eq. (7)): pair
    totals accumulated hyperedge by hyperedge over all vertex pairs."""
    h = generate(300, 320, 2, 12, 2.5, weights="lognormal", seed=12)
    R = np.diff(h.eptr).astype(np.float32)
    tot = {}
    for e in range(h.m):
        mem = [int(x) for x in h.pins[h.eptr[e]:h.eptr[e + 1]]]
        t = float(h.w[e]) / (len(mem) - 1)
        for a, b in itertools.permutations(mem, 2):
            tot[(a, b)] = tot.get((a, b), 0.0) + t
    best, val = ort.best_neighbours(h.n, h.m, h.eptr, h.pins, h.w, R, 1.0)
    for p in range(h.n):
        cand = {b: v for (a, b), v in tot.items() if a == p}
        if not cand:
            assert best[p] == -1 and val[p] == 0.0
            continue
        top = max(cand.values())
        assert val[p] == top
        assert best[p] == min(b for b, v in cand.items() if v == top)


def test_symmetric():
    h = generate(200, 220, 2, 10, 2.5, weights="lognormal", seed=13)
    R = np.random.default_rng(1).random(h.m).astype(np.float32)
    ne = ort.node_edges(h.n, h.eptr, h.pins)
    for p in range(0, h.n, 7):
        for q, v in ort.pair_ratings(p, ne[p], h.eptr, h.pins, h.w, R).items():
            back = ort.pair_ratings(q, ne[q], h.eptr, h.pins, h.w, R)[p]
            assert abs(v - back) <= 1e-12 * abs(v)
