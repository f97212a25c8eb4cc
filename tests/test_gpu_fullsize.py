"""Parity at the full configuration sizes, in the launch configuration the
benchmark times.

* netlist200k (200k nodes, 210k hyperedges, k = 20, b = 4) and large2m
  (2M nodes, 2.2M hyperedges, k = 30, b = 8): the FP32 estimate against the
  float64 oracle on 8192 sampled hyperedges and every Q_H value (stored by
  tests/golden/make_fullsize_samples.py, which calls only the oracle),
  within the FP32 bars (1e-4 norm-relative and at the 99.9th percentile
  over R >= 1e-3 max R; Q_H 1e-5).
* large2m (2M nodes, 2.2M hyperedges, k = 30, b = 8, 3 levels, the
  benchmark workload): properties that hold at any size -- the weighted
  ratios of every pool column sum to one (Eqs. (9), (13)), the pool is
  orthonormal, 0 <= R_e <= 1/w_e, hef_coarsen's level-0 R equals
  hef_resistance's, the cluster map is a canonical total surjection with
  eta >= 0, repeated runs are bitwise equal, and the BF16 pool stays within
  1e-2 of FP32.
* bf16_10m (10M nodes, 11M hyperedges, k = 30, b = 8, 3 levels, BF16 pool,
  the precision workload): the same properties, with the orthonormality
  bar of a bfloat16 basis (2e-2) and the BF16 estimate within 1e-2 of the
  FP32 one.  No oracle value exists at this size (a float64 pool would
  take 38 GB of host memory).
"""
import os

import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from synth import get_config, make_hypergraph
from tests.gpu_common import say, to_device

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _spread_sums(h, dh, chi, qh, chunk=32):
    """sum_e w_e (max - min)^2 / Q_H per column, on the device (float64)."""
    K = chi.shape[1]
    eptr = dh.eptr.long()
    sizes = (eptr[1:] - eptr[:-1])
    eid = torch.repeat_interleave(torch.arange(h.m, device="cuda"), sizes)
    w = dh.w.double()
    out = torch.empty(K, dtype=torch.float64, device="cuda")
    pins = dh.pins.long()
    for c0 in range(0, K, chunk):
        c1 = min(K, c0 + chunk)
        G = chi[pins, c0:c1].double()
        idx = eid[:, None].expand(-1, c1 - c0)
        mx = torch.full((h.m, c1 - c0), -np.inf, dtype=torch.float64, device="cuda")
        mn = torch.full((h.m, c1 - c0), np.inf, dtype=torch.float64, device="cuda")
        mx.scatter_reduce_(0, idx, G, reduce="amax")
        mn.scatter_reduce_(0, idx, G, reduce="amin")
        s = (mx - mn) ** 2
        out[c0:c1] = (w[:, None] * s).sum(0) / qh[c0:c1]
        del G, idx, mx, mn, s
    return out.cpu().numpy()


@pytest.mark.parametrize("name", ["netlist200k", "large2m"])
def test_matches_oracle_sample(name):
    cfg = get_config(name)
    h = make_hypergraph(name)
    ref = np.load(os.path.join(GOLD, f"{name}_R_sample.npz"))
    say(f"case: resistance {name} n={h.n} m={h.m} k={cfg['k']} b={cfg['b']}")
    dh = to_device(h)
    R, qh, _ = hef.resistance(dh, hef.Params(k=cfg["k"], b=cfg["b"], assume_valid=True))
    R = R.cpu().numpy().astype(np.float64)[ref["idx"]]
    Rref = ref["R"]
    norm = np.linalg.norm(R - Rref) / np.linalg.norm(Rref)
    nz = Rref >= 1e-3 * float(ref["Rmax"])
    rel = np.abs(R[nz] - Rref[nz]) / Rref[nz]
    qerr = np.abs(qh.cpu().numpy() - ref["qh"]).max() / ref["qh"].max()
    say(f"  sampled R norm-rel {norm:.2e} p99.9 {np.quantile(rel, 0.999):.2e} "
        f"max {rel.max():.2e}; qh {qerr:.2e}")
    assert norm <= 1e-4 and np.quantile(rel, 0.999) <= 1e-4
    assert qerr <= 1e-5


def test_large2m_properties_in_the_benchmark_configuration():
    cfg = get_config("large2m")
    h = make_hypergraph("large2m")
    say(f"case: large2m n={h.n} m={h.m} k={cfg['k']} b={cfg['b']} levels={cfg['levels']}")
    dh = to_device(h)
    p = hef.Params(k=cfg["k"], b=cfg["b"], levels=cfg["levels"], percentile=cfg["percentile"],
                   local_clustering=cfg["local_clustering"], assume_valid=True)
    R, qh, chi = hef.resistance(dh, hef.Params(k=cfg["k"], b=cfg["b"], assume_valid=True),
                                return_pool=True)
    a = hef.coarsen(dh, p)
    b = hef.coarsen(dh, p)
    say("  coarsen done twice")
    assert torch.equal(a[0], b[0]) and a[1] == b[1] and torch.equal(a[2], b[2])
    assert torch.equal(a[3], b[3])
    assert torch.equal(a[2], R)          # level 0 of Alg. 2 is Alg. 1
    w = dh.w
    Rc = R.double()
    assert bool(torch.isfinite(Rc).all()) and bool((Rc >= 0).all())
    assert bool((Rc * w.double() <= 1.0 + 1e-5).all())
    # orthonormal pool (float64 products of the float32 basis, row chunks)
    K = chi.shape[1]
    G = torch.zeros((K, K), dtype=torch.float64, device="cuda")
    for r0 in range(0, h.n, 250_000):
        blk = chi[r0:r0 + 250_000].double()
        G += blk.T @ blk
    orth = (G - torch.eye(K, dtype=torch.float64, device="cuda")).abs().max().item()
    say(f"  pool orthogonality {orth:.2e}")
    assert orth < 1e-4
    del G
    sums = _spread_sums(h, dh, chi, qh)
    say(f"  weighted ratio sums: max |1 - sum| {np.abs(sums - 1).max():.2e}")
    assert np.abs(sums - 1).max() < 1e-5
    cl, nc = a[0].cpu().numpy(), a[1]
    assert cl.min() == 0 and cl.max() == nc - 1 and np.unique(cl).size == nc
    first = np.full(nc, -1, dtype=np.int64)
    order = np.arange(h.n)[::-1]
    first[cl[order]] = order
    assert (np.diff(first) > 0).all()
    assert (a[3].cpu().numpy() >= 0).all()
    say(f"  clusters {nc} of {h.n}")
    # BF16 pool against FP32 at full size
    Rb, _, _ = hef.resistance(dh, hef.Params(k=cfg["k"], b=cfg["b"], basis="bf16",
                                             assume_valid=True))
    rb = (torch.linalg.norm(Rb.double() - Rc) / torch.linalg.norm(Rc)).item()
    say(f"  bf16 vs fp32 norm-rel {rb:.2e}")
    assert rb < 1e-2


def _canonical_map(cl, nc, n):
    assert cl.min() == 0 and cl.max() == nc - 1 and np.unique(cl).size == nc
    first = np.full(nc, -1, dtype=np.int64)
    order = np.arange(n)[::-1]
    first[cl[order]] = order
    assert (np.diff(first) > 0).all()


@pytest.mark.timeout(400)
def test_bf16_10m_properties():
    cfg = get_config("bf16_10m")
    h = make_hypergraph("bf16_10m")
    say(f"case: bf16_10m n={h.n} m={h.m} nnz={int(h.eptr[-1])} k={cfg['k']} b={cfg['b']} "
        f"levels={cfg['levels']} basis=bf16")
    dh = to_device(h)
    p = hef.Params(k=cfg["k"], b=cfg["b"], levels=cfg["levels"], percentile=cfg["percentile"],
                   local_clustering=cfg["local_clustering"], basis="bf16", assume_valid=True)
    a = hef.coarsen(dh, p)
    b = hef.coarsen(dh, p)
    say("  coarsen done twice")
    assert torch.equal(a[0], b[0]) and a[1] == b[1] and torch.equal(a[2], b[2])
    assert torch.equal(a[3], b[3])
    del b
    R, qh, chi = hef.resistance(dh, hef.Params(k=cfg["k"], b=cfg["b"], basis="bf16",
                                               assume_valid=True), return_pool=True)
    assert torch.equal(a[2], R)
    Rc = R.double()
    assert bool(torch.isfinite(Rc).all()) and bool((Rc >= 0).all())
    assert bool((Rc * dh.w.double() <= 1.0 + 1e-5).all())
    K = chi.shape[1]
    G = torch.zeros((K, K), dtype=torch.float64, device="cuda")
    for r0 in range(0, h.n, 1_000_000):
        blk = chi[r0:r0 + 1_000_000].double()
        G += blk.T @ blk
    orth = (G - torch.eye(K, dtype=torch.float64, device="cuda")).abs().max().item()
    say(f"  pool orthogonality {orth:.2e}")
    assert orth < 2e-2
    del G, blk
    sums = _spread_sums(h, dh, chi, qh, chunk=16)
    say(f"  weighted ratio sums: max |1 - sum| {np.abs(sums - 1).max():.2e}")
    assert np.abs(sums - 1).max() < 1e-5
    del chi
    _canonical_map(a[0].cpu().numpy(), a[1], h.n)
    assert (a[3].cpu().numpy() >= 0).all()
    say(f"  clusters {a[1]} of {h.n}")
    Rf, _, _ = hef.resistance(dh, hef.Params(k=cfg["k"], b=cfg["b"], assume_valid=True))
    rb = (torch.linalg.norm(Rc - Rf.double()) / torch.linalg.norm(Rf.double())).item()
    say(f"  bf16 vs fp32 norm-rel {rb:.2e}")
    assert rb < 1e-2
