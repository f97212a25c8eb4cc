"""GPU parity of Alg. 2 (a6-a10).

One level from GIVEN inputs (resistances, eta, pool, quadratic forms drawn
from the seeded generator, never from the GPU) must match the oracle bit for
bit: the node -> cluster map, the cluster count and every cluster's eta.  The
full coarsening (GPU resistances, so not bit-comparable with the FP64 oracle)
is checked for its invariants and its agreement is reported.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from oracle import clustering as ocl
from oracle import coarsen as oco
from synth import generate, make_hypergraph, start_block
from tests.gpu_common import say, to_device

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "cluster_level_examples.json")


def _gpu_level(h, R, eta, chi, qh, percentile=0.5, local=True):
    dh = to_device(h)
    K = chi.shape[1]
    params = hef.Params(k=K, b=1, star_only=True, percentile=percentile, local_clustering=local)
    assert params.K == K
    lab, nc, eta_out = hef.cluster_level(
        dh, params, torch.as_tensor(R, device="cuda"),
        None if eta is None else torch.as_tensor(eta, device="cuda"),
        torch.as_tensor(chi, device="cuda"), torch.as_tensor(qh, device="cuda"))
    return lab.cpu().numpy(), nc, eta_out.cpu().numpy()


def _check(h, R, eta, chi, qh, **kw):
    res = ocl.cluster_level(h.n, h.m, h.eptr, h.pins, R, eta, chi, qh, kw.get("percentile", 0.5),
                            kw.get("local", True))
    lab, nc, eta_out = _gpu_level(h, R, eta, chi, qh, **kw)
    say(f"  clusters: oracle {res.n_clusters} gpu {nc}; contracted {len(res.contracted)}, "
        f"attached {len(res.best)}")
    assert nc == res.n_clusters
    assert np.array_equal(lab, res.label)
    assert np.array_equal(eta_out.view(np.uint32), res.eta.view(np.uint32))


@pytest.mark.parametrize("ex", json.load(open(GOLD))["examples"], ids=lambda e: e["name"])
def test_hand_worked_levels(ex):
    say(f"case: cluster_level golden '{ex['name']}'")
    edges = ex["edges"]
    eptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])])
    pins = np.array([p for e in edges for p in e])
    from synth.hypergraph import Hypergraph
    h = Hypergraph(n=ex["n"], m=len(edges), eptr=eptr, pins=pins.astype(np.int32),
                   w=np.array(ex["w"], np.float32))
    R = np.array(ex["R"], np.float32)
    eta = np.array(ex["eta"], np.float32)
    chi = np.array(ex["chi"], np.float32)
    qh = np.array(ex["qh"], np.float64)
    lab, nc, eta_out = _gpu_level(h, R, eta, chi, qh)
    assert lab.tolist() == ex["expect_label"] and nc == ex["expect_n_clusters"]
    _check(h, R, eta, chi, qh)


def _inputs(h, K, seed, unusable=True):
    rng = np.random.default_rng(seed)
    R = rng.random(h.m).astype(np.float32)
    eta = (0.05 * rng.random(h.n)).astype(np.float32)
    chi = rng.standard_normal((h.n, K)).astype(np.float32)
    qh = rng.random(K) + 0.5
    if unusable:
        qh[1] = 0.0
    return R, eta, chi, qh


@pytest.mark.parametrize("local", [True, False])
def test_random_level_bit_exact(local):
    h = generate(3000, 3200, 2, 30, 2.5, p_loc=0.5, win=200, seed=41)
    say(f"case: cluster_level random n=3000 local={local}")
    _check(h, *_inputs(h, 6, 1), local=local)


def test_ties_in_resistance_and_distance():
    # quantised resistances and pool values force ties in both orders
    h = generate(2000, 2100, 2, 12, 2.5, p_loc=0.5, win=100, seed=43)
    rng = np.random.default_rng(3)
    R = (rng.integers(0, 8, h.m) / 8).astype(np.float32)
    chi = rng.integers(-2, 3, (h.n, 4)).astype(np.float32)
    qh = np.array([1.0, 2.0, 0.0, 4.0])
    say("case: cluster_level with ties")
    _check(h, R, None, chi, qh)
    _check(h, R, np.zeros(h.n, np.float32), chi, qh, percentile=0.3)


def test_no_isolated_node_and_only_isolated_nodes():
    # every node contracted (the best-neighbour list is empty), then a
    # threshold below every R (no contraction: every node is on the list)
    from synth.hypergraph import Hypergraph
    edges = [[0, 1], [2, 3], [1, 2], [4, 5, 6, 7]]
    eptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])])
    pins = np.array([p for e in edges for p in e], np.int32)
    h = Hypergraph(n=8, m=len(edges), eptr=eptr, pins=pins, w=np.ones(len(edges), np.float32))
    R = np.array([0.1, 0.2, 0.9, 0.3], np.float32)
    rng = np.random.default_rng(5)
    chi = rng.standard_normal((8, 3)).astype(np.float32)
    qh = np.array([1.0, 2.0, 0.5])
    say("case: cluster_level, all nodes contracted")
    _check(h, R, None, chi, qh, percentile=1.0)
    say("case: cluster_level, no contraction")
    _check(h, R, None, chi, qh, percentile=0.01)


def test_netlist_level_bit_exact():
    h = make_hypergraph("netlist200k")
    say(f"case: cluster_level netlist200k n={h.n} m={h.m} K=160")
    _check(h, *_inputs(h, 160, 2))


def test_coarsen_tiny_end_to_end():
    h = make_hypergraph("tiny2k")
    say("case: coarsen tiny2k k=10 b=1 levels=3")
    dh = to_device(h)
    cl, nc, R0, eta = hef.coarsen(dh, hef.Params(k=10, b=1, levels=3))
    cl = cl.cpu().numpy()
    start = lambda lev, x, rows, b: start_block(7, lev, x, rows, b).astype(np.float32).astype(np.float64)  # noqa: E731
    ref = oco.coarsen(h.n, h.m, h.eptr, h.pins, h.w, 10, 1, 3, start)
    rel = np.linalg.norm(R0.cpu().numpy() - ref.R0) / np.linalg.norm(ref.R0)
    same = (cl == ref.cluster).mean()
    say(f"  R0 norm-rel {rel:.2e}; clusters gpu {nc} oracle {ref.n_clusters}; "
        f"identical labels {same:.4f}")
    assert rel < 1e-4
    assert cl.min() == 0 and cl.max() == nc - 1 and np.unique(cl).size == nc
    first = np.array([np.nonzero(cl == c)[0].min() for c in range(nc)])
    assert (np.diff(first) > 0).all()
    assert eta.shape[0] == nc and (eta.cpu().numpy() >= 0).all()
    assert nc < h.n
    assert abs(nc - ref.n_clusters) <= 0.02 * ref.n_clusters


def test_coarsen_netlist_invariants_and_determinism():
    h = make_hypergraph("netlist200k")
    say("case: coarsen netlist200k k=20 b=4 levels=3")
    dh = to_device(h)
    p = hef.Params(k=20, b=4, levels=3)
    a = hef.coarsen(dh, p)
    b = hef.coarsen(dh, p)
    cl, nc = a[0].cpu().numpy(), a[1]
    say(f"  clusters {nc} (node reduction {1 - nc / h.n:.3f})")
    assert torch.equal(a[0], b[0]) and a[1] == b[1] and torch.equal(a[2], b[2])
    assert torch.equal(a[3], b[3])
    assert cl.min() == 0 and cl.max() == nc - 1 and np.unique(cl).size == nc
    assert nc < h.n


def _with_giant_edge(h, size):
    """h plus one more hyperedge over nodes 0 .. size-1 (weight 1)."""
    from synth.hypergraph import Hypergraph
    eptr = np.concatenate([h.eptr, [h.eptr[-1] + size]]).astype(h.eptr.dtype)
    pins = np.concatenate([h.pins, np.arange(size, dtype=h.pins.dtype)])
    w = np.concatenate([h.w, np.ones(1, h.w.dtype)])
    return Hypergraph(n=h.n, m=h.m + 1, eptr=eptr, pins=pins, w=w)


@pytest.mark.parametrize("giant", [0, 17000], ids=["sorted_per_hyperedge", "global_sort"])
def test_rebuild_matches_oracle_counts(giant):
    """Alg. 2's coarse rebuild on the GPU's own level-0 map: the coarse hypergraph the
    library builds for level 1 has the node, hyperedge and pin counts of the
    oracle's rebuild of the same map.  Hyperedges up to 16384 pins are sorted
    one per workgroup; the 17000-pin one sends the level to the global
    sort."""
    h = generate(40000, 30000, 2, 2000, 2.5, p_loc=0.6, win=300, weights="lognormal", seed=61)
    if giant:
        h = _with_giant_edge(h, giant)
    say(f"case: rebuild counts n={h.n} m={h.m} max|e|={h.sizes().max()}")
    dh = to_device(h)
    cl1, nc1, _, _ = hef.coarsen(dh, hef.Params(k=8, b=2, levels=1))
    m1, eptr1, pins1, _, _ = ocl.rebuild(h.m, h.eptr, h.pins, h.w, cl1.cpu().numpy())
    hef.coarsen(dh, hef.Params(k=8, b=2, levels=2))
    lev = hef.last_coarsen_levels()
    say(f"  level 1: gpu {lev[1]} oracle {(nc1, m1, int(eptr1[-1]))}")
    assert tuple(lev[1]) == (nc1, m1, int(eptr1[-1]))


def test_best_search_work_count():
    # with no contraction (delta is the smallest updated resistance and a
    # hyperedge contracts only strictly below it) every node with a
    # hyperedge is isolated, so the best-neighbour search screens one
    # candidate per co-pin occurrence: sum_e |e| (|e| - 1) at level 0
    h = make_hypergraph("tiny2k")
    dh = to_device(h)
    say("case: work count of the best-neighbour search, tiny2k")
    hef.coarsen(dh, hef.Params(k=10, b=1, levels=1, percentile=1e-9))
    w = hef.last_coarsen_work()
    sz = h.sizes().astype(np.int64)
    assert w == [int((sz * (sz - 1)).sum())]
    # the default threshold contracts part of the hyperedges: fewer, not none
    hef.coarsen(dh, hef.Params(k=10, b=1, levels=2))
    w2 = hef.last_coarsen_work()
    say(f"  counts {w} and {w2}")
    assert len(w2) == 2 and 0 < w2[0] < w[0]
    # without local clustering nothing is screened
    hef.coarsen(dh, hef.Params(k=10, b=1, levels=1, local_clustering=False))
    assert hef.last_coarsen_work() == [0]
