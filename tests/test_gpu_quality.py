"""GPU parity of the cluster-quality evaluator (Section II-A, Eq. (3);
Section IV, Eq. (18)) against the oracle.

Unit weights make every sum an integer, so cut, vol and phi must be equal
bit for bit.  With lognormal weights the two sides add the same positive
float64 terms in different orders: each sum of N terms is within (N - 1) u
(u = 2^-53) of the exact value, so the two differ by at most 2 N u relative;
phi adds one subtraction (vol(V) - vol(S), absolute error at most
4 nnz u vol(V)) and one division.  The tests use these bounds.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from oracle import quality as oq
from synth import generate, get_config, make_hypergraph
from synth.hypergraph import Hypergraph
from tests.gpu_common import say, to_device

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "conductance_examples.json")
U = 2.0 ** -53


def _gpu(h, label, nc):
    dh = to_device(h)
    cut, vol, phi, avg = hef.conductance(dh, torch.as_tensor(label.astype(np.int32),
                                                             device="cuda"), nc)
    return cut.cpu().numpy(), vol.cpu().numpy(), phi.cpu().numpy(), float(avg.item())


def _compare(h, label, nc, exact):
    cut, vol, phi, avg = _gpu(h, label, nc)
    rc, rv, rp = oq.cluster_conductance(h.n, h.eptr, h.pins, h.w, label, nc)
    ravg = oq.average_conductance(rp)
    say(f"  nc={nc}: phi_avg gpu {avg:.12f} oracle {ravg:.12f}")
    if exact:
        assert np.array_equal(cut, rc) and np.array_equal(vol, rv)
        assert np.array_equal(phi, rp)
        assert abs(avg - ravg) <= 2 * nc * U * max(ravg, 1e-300)
        return
    nnz = int(h.eptr[-1])
    tol = 2 * nnz * U
    np.testing.assert_allclose(cut, rc, rtol=tol, atol=0)
    np.testing.assert_allclose(vol, rv, rtol=tol, atol=0)
    total = rv.sum()
    den = np.minimum(rv, total - rv)
    ok = rc != 0
    ptol = np.zeros(nc)
    ptol[ok] = 4 * tol + 4 * nnz * U * total / den[ok]
    assert np.all(np.abs(phi - rp) <= ptol * np.maximum(rp, 0) + 1e-300)
    assert np.array_equal(phi == 0, rp == 0)
    assert abs(avg - ravg) <= (ptol.max() + 2 * nc * U) * ravg + 1e-300


_G = json.load(open(GOLD))


@pytest.mark.parametrize("ex", _G["examples"], ids=lambda e: e["name"])
def test_hand_worked(ex):
    say(f"case: conductance golden '{ex['name']}'")
    hg = _G["hypergraph"]
    edges = hg["edges"]
    eptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])])
    pins = np.array([p for e in edges for p in e], np.int32)
    h = Hypergraph(n=hg["n"], m=len(edges), eptr=eptr, pins=pins, w=np.array(hg["w"], np.float32))
    label = np.array(ex["label"])
    cut, vol, phi, avg = _gpu(h, label, max(ex["label"]) + 1)
    assert cut.tolist() == ex["cut"] and vol.tolist() == ex["vol"]
    np.testing.assert_allclose(phi, ex["phi"], rtol=1e-15, atol=0)
    assert abs(avg - ex["phi_avg"]) <= 1e-15


def _with_giant_edge(h, size):
    eptr = np.concatenate([h.eptr, [h.eptr[-1] + size]])
    pins = np.concatenate([h.pins, np.arange(size, dtype=h.pins.dtype)])
    w = np.concatenate([h.w, np.array([1.75], np.float32)]).astype(np.float32)
    return Hypergraph(n=h.n, m=h.m + 1, eptr=eptr, pins=pins, w=w)


@pytest.mark.parametrize("weights", ["unit", "lognormal"])
@pytest.mark.parametrize("nc", [1, 2, 37, 1000, 3000])
def test_random_partitions(weights, nc):
    say(f"case: conductance random weights={weights} nc={nc}")
    h = generate(3000, 3200, 2, 30, 2.5, p_loc=0.5, win=200, weights=weights, seed=17)
    if weights == "unit":
        h.w[:] = 1.0
    else:
        h = _with_giant_edge(h, 700)  # one cluster holds runs longer than a wave
    rng = np.random.default_rng(nc)
    label = rng.permutation(np.arange(h.n) % nc)
    _compare(h, label, nc, exact=weights == "unit")


def test_empty_clusters_and_nodes_without_hyperedges():
    say("case: conductance, unused labels and isolated nodes")
    h = generate(500, 400, 2, 12, 2.5, seed=3, weights="lognormal")
    deg = np.bincount(h.pins, minlength=h.n)
    say(f"  nodes without hyperedges: {(deg == 0).sum()}")
    rng = np.random.default_rng(4)
    label = 2 * rng.integers(0, 60, h.n)  # odd labels are empty
    _compare(h, label, 121, exact=False)


def test_partition_from_the_coarsening():
    say("case: conductance of a GPU coarsening (netlist-like, 20k nodes)")
    h = generate(20000, 21000, 2, 40, 2.5, p_loc=0.6, win=300, weights="lognormal", seed=5)
    cl, nc, _, _ = hef.coarsen(to_device(h), hef.Params(k=10, b=2, levels=2))
    _compare(h, cl.cpu().numpy(), nc, exact=False)


def test_no_hyperedges_and_errors():
    say("case: conductance edge cases and errors")
    h = Hypergraph(n=5, m=0, eptr=np.zeros(1, np.int64), pins=np.zeros(0, np.int32),
                   w=np.zeros(0, np.float32))
    cut, vol, phi, avg = _gpu(h, np.array([0, 1, 1, 2, 0]), 3)
    assert not cut.any() and not vol.any() and not phi.any() and avg == 0.0
    g = generate(300, 200, 2, 8, 2.5, seed=2)
    dh = to_device(g)
    lab = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(hef.HefError):
        hef.conductance(dh, lab, g.n + 1)
    with pytest.raises(hef.HefError):
        hef.conductance(dh, lab, 0)
    bad = lab.clone()
    bad[7] = 5
    with pytest.raises(hef.HefError):
        hef.conductance(dh, bad, 5)
    cut, vol, phi, avg = hef.conductance(dh, lab, 1)  # one cluster: no cut
    assert cut.item() == 0.0 and phi.item() == 0.0 and avg.item() == 0.0


@pytest.mark.timeout(400)
def test_large2m_sampled_clusters():
    cfg = get_config("large2m")
    h = make_hypergraph("large2m")
    say(f"case: conductance large2m n={h.n} m={h.m}")
    dh = to_device(h)
    p = hef.Params(k=cfg["k"], b=cfg["b"], levels=cfg["levels"], percentile=cfg["percentile"],
                   local_clustering=cfg["local_clustering"], assume_valid=True)
    cl, nc, _, _ = hef.coarsen(dh, p)
    cut, vol, phi, avg = hef.conductance(dh, cl, nc)
    cut, vol, phi = cut.cpu().numpy(), vol.cpu().numpy(), phi.cpu().numpy()
    avg = float(avg.item())
    label = cl.cpu().numpy()
    w64 = h.w.astype(np.float64)
    total = float((w64 * np.diff(h.eptr)).sum())
    nnz = int(h.eptr[-1])
    say(f"  clusters {nc}, phi_avg {avg:.6f}")
    assert abs(vol.sum() - total) <= 4 * nnz * U * total
    assert np.all(phi >= 0) and np.all(phi <= 1 + 1e-12)
    assert abs(avg - phi.mean()) <= 4 * nc * U * avg
    rng = np.random.default_rng(11)
    for c in rng.choice(nc, 48, replace=False):
        oc, ov = oq.one_cluster(h.eptr, h.pins, h.w, label, c)
        assert abs(cut[c] - oc) <= 2 * nnz * U * oc
        assert abs(vol[c] - ov) <= 2 * nnz * U * ov
        ref = 0.0 if oc == 0 else oc / min(ov, total - ov)
        assert abs(phi[c] - ref) <= 16 * nnz * U * max(ref, 1e-300)
