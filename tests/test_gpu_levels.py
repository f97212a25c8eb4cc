"""GPU parity of the level hand-off of Alg. 2 (steps 4-10 and the coarse
rebuild of step 6) on the path the coarsening itself runs.

* One level fed with the library's own K = 480 pool (FP32 and BF16 storage:
  orthonormal magnitudes, every column stage of the best-neighbour screen),
  against the oracle given the same R, chi and Q_H: labels, count and eta
  bit for bit.
* The coarse hypergraph of hef_rebuild against the oracle's rebuild element
  by element (the per-hyperedge sorts and the global-sort path).
* A chain of levels on the GPU (Alg. 1 with the level's start blocks, one
  clustering level, rebuild) against the oracle chain fed the GPU's R, chi
  and Q_H per level, and against hef_coarsen_levels' own per-level record
  and final map, bit for bit.
* The node-reduction stop rule of the level loop.
"""
import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from oracle import clustering as ocl
from synth import generate, make_hypergraph
from synth.hypergraph import Hypergraph
from tests.gpu_common import say, to_device

pytestmark = pytest.mark.gpu


def _np64(chi):
    return chi.float().cpu().numpy().astype(np.float64)


def _host(dh):
    """A DeviceHypergraph back on the host (int64 CSR, float32 w)."""
    return Hypergraph(n=dh.n, m=dh.m, eptr=dh.eptr.cpu().numpy().astype(np.int64),
                      pins=dh.pins.cpu().numpy().astype(np.int64),
                      w=dh.w.cpu().numpy().astype(np.float32))


def _same_bits(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))


@pytest.mark.parametrize("basis", ["fp32", "bf16"])
def test_k480_level_from_the_librarys_pool(basis):
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=5)
    dh = to_device(h)
    p = hef.Params(k=30, b=8, basis=basis)
    R, qh, chi = hef.resistance(dh, p, return_pool=True)
    say(f"case: cluster_level K={p.K} ({basis} pool from hef_resistance) n={h.n} m={h.m}; "
        f"max |chi| {float(chi.float().abs().max()):.3e}")
    lab, nc, eta = hef.cluster_level(dh, p, R, None, chi, qh)
    res = ocl.cluster_level(h.n, h.m, h.eptr, h.pins, R.cpu().numpy(), None, _np64(chi),
                            qh.cpu().numpy(), 0.5, True)
    say(f"  clusters gpu {nc} oracle {res.n_clusters}; attached {len(res.best)}")
    assert p.K > 256  # the screen's third column stage runs
    assert nc == res.n_clusters
    assert np.array_equal(lab.cpu().numpy(), res.label)
    assert _same_bits(eta.cpu().numpy(), res.eta)


def test_pool_outside_float16_range_is_rejected():
    h = make_hypergraph("tiny2k")
    dh = to_device(h)
    p = hef.Params(k=10, b=1)
    R, qh, chi = hef.resistance(dh, p, return_pool=True)
    for bad in (7.0e4, float("nan"), float("inf")):
        say(f"case: cluster_level with a pool value {bad}")
        c = chi.clone()
        c[17, 3] = bad
        with pytest.raises(hef.HefError) as ei:
            hef.cluster_level(dh, p, R, None, c, qh)
        assert ei.value.status == 1
    # without local clustering the pool is not read
    lab, nc, _ = hef.cluster_level(dh, hef.Params(k=10, b=1, local_clustering=False), R, None,
                                   c, qh)
    assert nc > 0


def _with_giant_edge(h, size):
    eptr = np.concatenate([h.eptr, [h.eptr[-1] + size]]).astype(h.eptr.dtype)
    pins = np.concatenate([h.pins, np.arange(size, dtype=h.pins.dtype)])
    w = np.concatenate([h.w, np.ones(1, h.w.dtype)])
    return Hypergraph(n=h.n, m=h.m + 1, eptr=eptr, pins=pins, w=w)


@pytest.mark.parametrize("giant", [0, 17000], ids=["sorted_per_hyperedge", "global_sort"])
def test_rebuild_elementwise(giant):
    h = generate(40000, 30000, 2, 2000, 2.5, p_loc=0.6, win=300, weights="lognormal", seed=61)
    if giant:
        h = _with_giant_edge(h, giant)
    say(f"case: hef_rebuild n={h.n} m={h.m} max|e|={h.sizes().max()}")
    dh = to_device(h)
    cl, nc, _, _ = hef.coarsen(dh, hef.Params(k=8, b=2, levels=1))
    h2, kept = hef.rebuild(dh, cl, nc)
    m2, eptr2, pins2, w2, kept_ref = ocl.rebuild(h.m, h.eptr, h.pins, h.w, cl.cpu().numpy())
    say(f"  coarse: gpu (n={h2.n}, m={h2.m}, nnz={h2.nnz}) oracle (m={m2}, nnz={int(eptr2[-1])})")
    assert h2.m == m2 and h2.n == nc
    assert np.array_equal(h2.eptr.cpu().numpy(), eptr2)
    assert np.array_equal(h2.pins.cpu().numpy(), pins2)
    assert _same_bits(h2.w.cpu().numpy(), np.asarray(w2, np.float32))
    assert np.array_equal(kept.cpu().numpy(), kept_ref)


def test_rebuild_rejects_bad_labels():
    h = make_hypergraph("tiny2k")
    dh = to_device(h)
    lab = torch.zeros(h.n, dtype=torch.int32, device="cuda")
    lab[h.pins[5]] = 3
    say("case: hef_rebuild with a label outside [0, n_clusters)")
    with pytest.raises(hef.HefError) as ei:
        hef.rebuild(dh, lab, 2)
    assert ei.value.status == 1


CHAINS = [("tiny2k", None, 10, 1, 3), ("netlist20k", 5, 30, 8, 2)]


@pytest.mark.parametrize("chain", CHAINS, ids=[c[0] for c in CHAINS])
def test_level_chain_bit_exact(chain):
    name, seed, k, b, levels = chain
    h = (make_hypergraph("tiny2k") if name == "tiny2k" else
         generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=seed))
    say(f"case: level chain {name} n={h.n} m={h.m} k={k} b={b} levels={levels}")
    p = hef.Params(k=k, b=b)
    dh = to_device(h)
    gmap = torch.arange(h.n, dtype=torch.int32, device="cuda")
    omap = np.arange(h.n)
    eta_g = None
    oh, eta_o = h, None
    chain_R, chain_lab, chain_eta = [], [], []
    for lev in range(levels):
        xs = hef.start_block(p.seed, lev, 0, dh.n + dh.m, b)
        xc = hef.start_block(p.seed, lev, 1, dh.n, b)
        R, qh, chi = hef.resistance(dh, p, xs, xc, return_pool=True)
        lab, nc, eta = hef.cluster_level(dh, p, R, eta_g, chi, qh)
        res = ocl.cluster_level(oh.n, oh.m, oh.eptr, oh.pins, R.cpu().numpy(), eta_o, _np64(chi),
                                qh.cpu().numpy(), 0.5, True)
        say(f"  level {lev}: n={dh.n} m={dh.m} -> gpu {nc} oracle {res.n_clusters}")
        assert nc == res.n_clusters
        assert np.array_equal(lab.cpu().numpy(), res.label)
        assert _same_bits(eta.cpu().numpy(), res.eta)
        chain_R.append(R)
        chain_lab.append(lab)
        chain_eta.append(eta)
        gmap = lab[gmap.long()]
        omap = res.label[omap]
        dh2, kept = hef.rebuild(dh, lab, nc)
        m2, eptr2, pins2, w2, kept_ref = ocl.rebuild(oh.m, oh.eptr, oh.pins, oh.w, res.label)
        assert dh2.m == m2
        assert np.array_equal(dh2.eptr.cpu().numpy(), eptr2)
        assert np.array_equal(dh2.pins.cpu().numpy(), pins2)
        assert np.array_equal(kept.cpu().numpy(), kept_ref)
        dh, eta_g = dh2, eta
        oh = Hypergraph(n=nc, m=m2, eptr=eptr2, pins=pins2.astype(np.int64),
                        w=np.asarray(w2, np.float32))
        eta_o = res.eta
        if dh.m == 0:
            break
    assert np.array_equal(gmap.cpu().numpy(), omap)
    # the library's own level loop: the same levels, bit for bit
    cl, nc, R0, eta, lv = hef.coarsen_levels(to_device(h), hef.Params(k=k, b=b, levels=levels))
    rho_min = [float(x["rho"][x["rho"] > 0].min()) for x in lv]
    say(f"  hef_coarsen_levels: {len(lv)} levels, {nc} clusters; min rho per level {rho_min}")
    assert len(lv) == len(chain_R)
    assert torch.equal(cl, gmap) and nc == int(gmap.max()) + 1
    assert torch.equal(eta, chain_eta[-1])
    assert torch.equal(R0, chain_R[0])
    for x, R, lab, e in zip(lv, chain_R, chain_lab, chain_eta):
        assert torch.equal(x["R"], R) and torch.equal(x["label"], lab) and torch.equal(x["eta"], e)
        kept = x["rho"][x["rho"] > 0]
        assert kept.numel() > 0 and float(kept.min()) > 1e-3 and float(kept.max()) <= 1.0 + 1e-12
    # hef_coarsen (no record) gives the same map
    cl2, nc2, _, eta2 = hef.coarsen(to_device(h), hef.Params(k=k, b=b, levels=levels))
    assert torch.equal(cl2, cl) and nc2 == nc and torch.equal(eta2, eta)


@pytest.mark.parametrize("nr", [0.6, 0.8])
def test_node_reduction_target(nr):
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=9)
    say(f"case: coarsen_levels with target_nr={nr} (cap 12 levels) n={h.n}")
    cap = 12
    cl, nc, _, _, lv = hef.coarsen_levels(to_device(h), hef.Params(k=10, b=4, levels=cap,
                                                                   target_nr=nr))
    goal = (1.0 - float(np.float32(nr))) * h.n
    ns = [x["n"] for x in lv] + [nc]
    say(f"  node counts per level {ns}, goal <= {goal:.0f}")
    for x in lv:
        assert x["n"] > goal                        # a level runs only while above the goal
    stalled = len(ns) >= 2 and ns[-1] == ns[-2]
    assert nc <= goal or len(lv) == cap or stalled
    assert np.unique(cl.cpu().numpy()).size == nc
    # the same run with a fixed level count of len(lv) gives the same map
    cl2, nc2, _, _ = hef.coarsen(to_device(h), hef.Params(k=10, b=4, levels=len(lv)))
    assert torch.equal(cl, cl2) and nc == nc2
