"""Pins of the conductance oracle (Section II-A, Eq. (3); Eq. (18)).

* hand-worked values (tests/golden/conductance_examples.json);
* on a 2-uniform hypergraph (a simple graph) the cut of a set S is
  x^T L x for its indicator x and the graph Laplacian L, and the degrees are
  the adjacency row sums (scipy.sparse, not the oracle's loops);
* a two-cluster partition has equal conductances (the cut and the smaller
  volume are shared);
* the volumes add up to sum_e w(e)|e|, and 0 <= phi <= 1;
* the cut of every cluster equals the weight of the hyperedges with some
  but not all pins in it (a count per hyperedge, not a set of labels).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import quality as oq
from synth import generate

GOLD = os.path.join(os.path.dirname(__file__), "golden", "conductance_examples.json")


def _arrays(edges):
    eptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    pins = np.array([p for e in edges for p in e], dtype=np.int64)
    return eptr, pins


_G = json.load(open(GOLD))


@pytest.mark.parametrize("ex", _G["examples"], ids=lambda e: e["name"])
def test_hand_worked(ex):
    hg = _G["hypergraph"]
    eptr, pins = _arrays(hg["edges"])
    nc = max(ex["label"]) + 1
    cut, vol, phi = oq.cluster_conductance(hg["n"], eptr, pins, np.array(hg["w"]),
                                           np.array(ex["label"]), nc)
    np.testing.assert_allclose(cut, ex["cut"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(vol, ex["vol"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(phi, ex["phi"], rtol=1e-15, atol=0)
    assert abs(oq.average_conductance(phi) - ex["phi_avg"]) <= 1e-15


def test_degrees_hand_worked():
    hg = _G["hypergraph"]
    eptr, pins = _arrays(hg["edges"])
    d = oq.degrees(hg["n"], eptr, pins, np.array(hg["w"]))
    assert d.tolist() == [1.5, 2.0, 4.0, 3.0, 1.0, 1.5, 0.0]


def test_graph_cut_is_laplacian_quadratic_form():
    rng = np.random.default_rng(3)
    n, m = 60, 150
    pairs = set()
    while len(pairs) < m:
        u, v = rng.integers(0, n, 2)
        if u != v:
            pairs.add((min(u, v), max(u, v)))
    edges = sorted(pairs)
    w = rng.random(m) + 0.25
    eptr, pins = _arrays(edges)
    u = np.array([e[0] for e in edges])
    v = np.array([e[1] for e in edges])
    A = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                      shape=(n, n)).tocsr()
    deg = np.asarray(A.sum(axis=1)).ravel()
    L = sp.diags(deg) - A
    nc = 5
    label = rng.integers(0, nc, n)
    cut, vol, phi = oq.cluster_conductance(n, eptr, pins, w, label, nc)
    for c in range(nc):
        x = (label == c).astype(np.float64)
        assert cut[c] == pytest.approx(x @ (L @ x), rel=1e-13)
        assert vol[c] == pytest.approx(x @ deg, rel=1e-13)
        den = min(vol[c], deg.sum() - vol[c])
        assert phi[c] == pytest.approx(0.0 if cut[c] == 0 else cut[c] / den, rel=1e-13)


def test_two_clusters_share_their_conductance():
    h = generate(400, 500, 2, 12, 2.5, p_loc=0.5, win=50, seed=8)
    rng = np.random.default_rng(1)
    label = rng.integers(0, 2, h.n)
    cut, vol, phi = oq.cluster_conductance(h.n, h.eptr, h.pins, h.w, label, 2)
    assert cut[0] == cut[1] > 0
    assert phi[0] == phi[1]


@pytest.mark.parametrize("nc", [1, 3, 40, 400])
def test_volume_total_bounds_and_per_edge_cut(nc):
    h = generate(400, 500, 2, 12, 2.5, p_loc=0.5, win=50, weights="lognormal", seed=9)
    rng = np.random.default_rng(nc)
    label = rng.permutation(np.arange(h.n) % nc)
    cut, vol, phi = oq.cluster_conductance(h.n, h.eptr, h.pins, h.w, label, nc)
    sizes = np.diff(h.eptr)
    assert vol.sum() == pytest.approx(float((h.w.astype(np.float64) * sizes).sum()), rel=1e-13)
    assert np.all(phi >= 0) and np.all(phi <= 1 + 1e-15)
    for c in range(nc):
        inside = np.add.reduceat((label[h.pins] == c).astype(np.int64), h.eptr[:-1])
        split = (inside > 0) & (inside < sizes)
        assert cut[c] == pytest.approx(float(h.w[split].astype(np.float64).sum()), rel=1e-13,
                                       abs=0)
        oc, ov = oq.one_cluster(h.eptr, h.pins, h.w, label, c)
        assert oc == pytest.approx(cut[c], rel=1e-13, abs=0)
        assert ov == pytest.approx(vol[c], rel=1e-13, abs=0)
    if nc == 1:
        assert cut[0] == 0 and phi[0] == 0


def test_planted_mistake_double_count_is_caught():
    # counting a split hyperedge once per pin instead of once per cluster
    # changes the hand-worked cut of the three-pair example
    hg = _G["hypergraph"]
    eptr, pins = _arrays(hg["edges"])
    label = np.array(_G["examples"][1]["label"])
    w = np.array(hg["w"])
    wrong = np.zeros(4)
    for e in range(len(w)):
        labs = label[pins[eptr[e]:eptr[e + 1]]]
        if len(set(labs.tolist())) > 1:
            for c in labs:
                wrong[c] += w[e]
    assert wrong.tolist() != _G["examples"][1]["cut"]
