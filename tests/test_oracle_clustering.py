"""Pins of the oracle's Alg. 2 level: hand-worked examples, invariants of the
greedy contraction, library union-find, brute-force nearest clusters, and
structural invariants of the coarse hypergraph."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from oracle import clustering as ocl
from oracle import coarsen as oco
from synth import generate, make_hypergraph, start_block

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cluster_level_examples.json")


def _csr(edges):
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    pins = np.array([p for e in edges for p in e], dtype=np.int64)
    return eptr, pins


@pytest.mark.parametrize("ex", json.load(open(GOLD))["examples"], ids=lambda e: e["name"])
def test_hand_worked_levels(ex):
    n = ex["n"]
    eptr, pins = _csr(ex["edges"])
    m = len(ex["edges"])
    R = np.array(ex["R"], dtype=np.float32)
    eta = np.array(ex["eta"], dtype=np.float32)
    chi = np.array(ex["chi"], dtype=np.float32)
    qh = np.array(ex["qh"], dtype=np.float64)
    res = ocl.cluster_level(n, m, eptr, pins, R, eta, chi, qh, ex["percentile"], True)
    # Eq. (15) by the example's own arithmetic
    R_upd = np.array([np.float32(sum(float(eta[v]) for v in e) + float(R[j]))
                      for j, e in enumerate(ex["edges"])], dtype=np.float32)
    assert np.array_equal(res.R_upd, R_upd)
    assert res.delta == float(R_upd[ex["expect_delta_edge"]])
    assert res.contracted == ex["expect_contracted"]
    assert res.label.tolist() == ex["expect_label"]
    assert res.n_clusters == ex["expect_n_clusters"]
    for c, terms in enumerate(ex["expect_eta_terms"]):
        acc = 0.0
        for t in terms:
            if isinstance(t, str) and t.startswith("eta"):
                acc += float(eta[int(t[3:])])
            elif isinstance(t, str) and t.startswith("R"):
                acc += float(R_upd[int(t[1:])])
            else:
                acc += float(t)
        assert res.eta[c] == np.float32(acc), (c, res.eta[c], acc)
    m2, eptr2, pins2, w2, kept = ocl.rebuild(m, eptr, pins, np.array(ex["w"], np.float32), res.label)
    got = [pins2[eptr2[j]:eptr2[j + 1]].tolist() for j in range(m2)]
    assert got == ex["expect_coarse_edges"]
    assert kept.tolist() == ex["expect_kept"]


def _random_level(seed, n=3000, m=3200, K=6, local=True):
    h = generate(n, m, 2, 30, 2.5, p_loc=0.5, win=200, seed=seed)
    rng = np.random.default_rng(seed)
    R = rng.random(h.m).astype(np.float32)
    eta = (0.1 * rng.random(h.n)).astype(np.float32)
    chi = rng.standard_normal((h.n, K)).astype(np.float32)
    qh = rng.random(K) + 0.5
    qh[1] = 0.0                                   # an unusable column
    res = ocl.cluster_level(h.n, h.m, h.eptr, h.pins, R, eta, chi, qh, 0.5, local)
    return h, R, eta, chi, qh, res


def test_greedy_contraction_invariants():
    h, R, eta, chi, qh, res = _random_level(1)
    R_upd = res.R_upd
    taken = np.full(h.n, -1)
    for e in res.contracted:
        mem = h.pins[h.eptr[e]:h.eptr[e + 1]]
        assert R_upd[e] < res.delta
        assert (taken[mem] < 0).all()            # pairwise disjoint
        taken[mem] = e
    cset = set(res.contracted)
    key = lambda e: (R_upd[e], e)                # noqa: E731
    for e in range(h.m):
        if R_upd[e] < res.delta and e not in cset:
            mem = h.pins[h.eptr[e]:h.eptr[e + 1]]
            blockers = taken[mem][taken[mem] >= 0]
            # maximal: blocked by a contracted hyperedge that comes earlier
            assert blockers.size and min(key(b) for b in blockers) < key(e)
    # the threshold admits at most ceil(pi m) - 1 hyperedges
    assert (R_upd < res.delta).sum() <= int(np.ceil(0.5 * h.m)) - 1


def test_local_clustering_matches_brute_force_and_union_find():
    h, R, eta, chi, qh, res = _random_level(2)
    n = h.n
    # provisional labels from the contraction
    prov = np.arange(n)
    for e in res.contracted:
        mem = h.pins[h.eptr[e]:h.eptr[e + 1]]
        prov[mem] = mem.min()
    single = np.ones(n, bool)
    for e in res.contracted:
        single[h.pins[h.eptr[e]:h.eptr[e + 1]]] = False
    members = {}
    for v in range(n):
        members.setdefault(int(prov[v]), []).append(v)
    use = qh > 0
    chi64 = chi.astype(np.float64)
    for p, c in list(res.best.items())[:400]:
        assert single[p]
        cands = set()
        for e in range(h.m):
            mem = h.pins[h.eptr[e]:h.eptr[e + 1]]
            if p in mem:
                cands |= {int(prov[v]) for v in mem if v != p}
        dists = {}
        for cl in cands:
            cen = np.zeros(chi.shape[1])
            for v in sorted(members[cl]):
                cen = cen + chi64[v]
            cen = cen / len(members[cl])
            diffs = [chi64[p, i] - cen[i] for i in np.nonzero(use)[0]]
            dists[cl] = max(d * d / qh[i] for d, i in zip(diffs, np.nonzero(use)[0]))
        dmin = min(dists.values())
        assert c == min(cl for cl, d in dists.items() if d == dmin)
        assert res.dist[p] == dmin
    # union-find equals the connected components of the attach graph
    labs = np.unique(prov)
    idx = {int(l): i for i, l in enumerate(labs)}
    rows = [idx[p] for p in res.best]
    cols = [idx[c] for c in res.best.values()]
    G = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(labs.size, labs.size))
    ncomp, comp = connected_components(G, directed=False)
    assert ncomp == res.n_clusters
    lab_of_prov = res.label[labs]
    for a in range(labs.size):
        for bq in (a + 1, (a * 7) % labs.size):
            if bq < labs.size:
                assert (comp[a] == comp[bq]) == (lab_of_prov[a] == lab_of_prov[bq])


def test_labels_are_canonical_and_total():
    h, R, eta, chi, qh, res = _random_level(3)
    lab = res.label
    assert lab.min() == 0 and lab.max() == res.n_clusters - 1
    assert np.unique(lab).size == res.n_clusters           # surjection onto [0, C)
    first = np.array([np.nonzero(lab == c)[0].min() for c in range(res.n_clusters)])
    assert (np.diff(first) > 0).all()                      # rank of smallest member id
    assert res.eta.shape == (res.n_clusters,) and (res.eta >= 0).all()


def test_no_local_clustering_leaves_singletons():
    h, R, eta, chi, qh, res = _random_level(4, local=False)
    assert not res.best
    single = np.ones(h.n, bool)
    for e in res.contracted:
        single[h.pins[h.eptr[e]:h.eptr[e + 1]]] = False
    assert res.n_clusters == single.sum() + len(res.contracted)
    # singletons keep their eta
    for v in np.nonzero(single)[0][:50]:
        assert res.eta[res.label[v]] == eta[v]


def test_rebuild_invariants():
    h, R, eta, chi, qh, res = _random_level(5)
    m2, eptr2, pins2, w2, kept = ocl.rebuild(h.m, h.eptr, h.pins, h.w, res.label)
    assert (np.diff(eptr2) >= 2).all()
    for j, e in enumerate(kept):
        img = np.unique(res.label[h.pins[h.eptr[e]:h.eptr[e + 1]]])
        assert np.array_equal(pins2[eptr2[j]:eptr2[j + 1]], img)
        assert w2[j] == h.w[e]
    dropped = np.setdiff1d(np.arange(h.m), kept)
    for e in dropped[:200]:
        assert np.unique(res.label[h.pins[h.eptr[e]:h.eptr[e + 1]]]).size < 2


def test_multilevel_coarsening_shrinks_and_composes():
    h = make_hypergraph("tiny2k")
    start = lambda lev, x, rows, b: start_block(7, lev, x, rows, b)  # noqa: E731
    out = oco.coarsen(h.n, h.m, h.eptr, h.pins, h.w, 6, 1, 3, start)
    assert len(out.levels) == 3
    ns = [lv[0] for lv in out.levels] + [out.n_clusters]
    assert all(a > b for a, b in zip(ns, ns[1:]))
    assert np.unique(out.cluster).size == out.n_clusters
    assert out.cluster.min() == 0 and out.cluster.max() == out.n_clusters - 1
    assert out.eta.shape == (out.n_clusters,)
    assert (out.eta >= 0).all()
    assert out.R0.shape == (h.m,)


GOLD2 = os.path.join(os.path.dirname(__file__), "golden", "coarsen_two_level_examples.json")


@pytest.mark.parametrize("ex", json.load(open(GOLD2))["examples"], ids=lambda e: e["name"])
def test_hand_worked_two_level_coarsening(ex, monkeypatch):
    """The level loop of Alg. 2 with prescribed per-level resistances: the
    composed map, the eta carried into the next level's Eq. (15), and the
    final eta, against hand-worked values."""
    from types import SimpleNamespace

    calls = []

    def fake_resistance(n, m, eptr, pins, w, Xs, Xc, k, tau=1e-3, **kw):
        lev = ex["levels"][len(calls)]
        calls.append((n, m, int(np.asarray(eptr)[-1])))
        assert len(lev["R"]) == m and len(lev["chi"]) == n
        return SimpleNamespace(R=np.array(lev["R"], dtype=np.float32),
                               qh=np.array(lev["qh"], dtype=np.float64),
                               pool=SimpleNamespace(chi=np.array(lev["chi"], dtype=np.float64)))

    monkeypatch.setattr(oco.resistance, "resistance", fake_resistance)
    eptr, pins = _csr(ex["edges"])
    start = lambda lev, x, rows, b: np.zeros((rows, b))  # noqa: E731
    out = oco.coarsen(ex["n"], len(ex["edges"]), eptr, pins, np.array(ex["w"], np.float32), 1, 1,
                      len(ex["levels"]), start, 0.5, ex["local_clustering"])
    assert [list(c) for c in calls] == ex["expect_level_sizes"]
    assert out.cluster.tolist() == ex["expect_cluster"]
    assert out.n_clusters == ex["expect_n_clusters"]
    # level-0 R_upd is R itself (eta = 0); level-1 R_upd adds the eta of the
    # level-0 clusters in CSR pin order (float64, then float32)
    lev0, lev1 = out.levels[0][3], out.levels[1][3]
    assert np.array_equal(lev0.R_upd, np.array(ex["expect_R_upd"][0], dtype=np.float32))
    eta1 = lev0.eta
    for j, terms in enumerate(ex["expect_R_upd"][1]):
        acc = 0.0
        for t in terms[1:]:
            acc += float(eta1[int(t[3:])]) if isinstance(t, str) else float(np.float32(t))
        assert lev1.R_upd[j] == np.float32(acc), (j, lev1.R_upd[j], acc)
    if ex.get("expect_level_eta"):
        first = ex["expect_level_eta"][0]
        assert lev0.eta[0] == np.float32(first[0])
        assert lev0.eta[1] == np.float32(sum([float(np.float32(first[1][0]))] + first[1][1:]))
    exp = ex["expect_eta"]
    if exp and isinstance(exp[0], list):
        # final eta as a sum of level-1 cluster etas and attach distances
        for c, terms in enumerate(exp[0]):
            acc = 0.0
            for t in terms:
                acc += float(lev0.eta[int(t[8:])]) if isinstance(t, str) else float(t)
            assert out.eta[c] == np.float32(acc), (c, out.eta[c], acc)
    else:
        assert np.array_equal(out.eta, np.array(exp, dtype=np.float32))


def test_node_reduction_target_stops_the_level_loop(monkeypatch):
    """Section IV's NR target on the hand-worked two-level example: level 0
    takes 6 nodes to 4.  NR = 0.3 (goal 4.2 nodes) stops after level 0;
    NR = 0.5 (goal 3) runs level 1 (4 -> 3 nodes) and stops there, below the
    cap of 5 levels; NR = 0.9 (goal 0.6) runs on until a level merges
    nothing.  Levels past the second reuse the second level's R prefix."""
    from types import SimpleNamespace
    ex = json.load(open(GOLD2))["examples"][0]

    def fake_resistance(n, m, eptr, pins, w, Xs, Xc, k, tau=1e-3, **kw):
        lev = ex["levels"][min(len(calls), 1)]
        calls.append(n)
        R = np.array(lev["R"][:m] + [0.5] * max(0, m - len(lev["R"])), dtype=np.float32)
        return SimpleNamespace(R=R, qh=np.ones(1), pool=SimpleNamespace(chi=np.zeros((n, 1))))

    monkeypatch.setattr(oco.resistance, "resistance", fake_resistance)
    eptr, pins = _csr(ex["edges"])
    start = lambda lev, x, rows, b: np.zeros((rows, b))  # noqa: E731
    run = lambda nr: oco.coarsen(ex["n"], len(ex["edges"]), eptr, pins,  # noqa: E731
                                 np.ones(len(ex["edges"]), np.float32), 1, 1, 5, start, 0.5,
                                 False, target_nr=nr)
    calls = []
    out = run(0.3)
    assert calls == [6] and out.n_clusters == 4
    calls = []
    out = run(0.5)
    assert calls == [6, 4] and out.n_clusters == 3
    # NR = 0.9: level 2 (edges {0,1} {1,2} {0,2}, R_upd 0.31 0.26 0.41,
    # delta 0.31) merges {1,2}; level 3 (two copies of {0,1}, R_upd 0.37
    # 0.41, delta 0.37) merges nothing, and the loop stops there
    calls = []
    out = run(0.9)
    assert calls == [6, 4, 3, 2] and out.n_clusters == 2
