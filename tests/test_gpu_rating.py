"""GPU parity of the Eq. (17) vertex-pair rating (hef_rating) against the
oracle, bit for bit (float64 sums in ascending hyperedge order on both
sides): resistances from the library's own estimate with both readings of
the denominator, the Eq. (7) special case, hub nodes and a hyperedge of 3000
pins, a batched run, and the error paths."""
import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from oracle import rating as ort
from synth import generate
from synth.hypergraph import Hypergraph
from tests.gpu_common import say, to_device

pytestmark = pytest.mark.gpu


def _check(h, R, shift, nodes=None):
    dh = to_device(h)
    best, val = hef.rating(dh, torch.as_tensor(R, device="cuda"), shift)
    best, val = best.cpu().numpy(), val.cpu().numpy()
    rb, rv = ort.best_neighbours(h.n, h.m, h.eptr, h.pins, h.w, R, shift, nodes)
    if nodes is not None:
        best, val = best[nodes], val[nodes]
    say(f"  shift={shift}: {int((best >= 0).sum())} nodes with neighbours; "
        f"rating range [{val.min():.3e}, {val.max():.3e}]")
    assert np.array_equal(best, rb)
    assert np.array_equal(val.view(np.uint64), rv.view(np.uint64))


def _with_hubs(h, seed):
    rng = np.random.default_rng(seed)
    edges = [list(h.pins[h.eptr[e]:h.eptr[e + 1]]) for e in range(h.m)]
    for hub in (11, 5000, 9999):
        for e in rng.choice(h.m, size=300, replace=False):
            if hub not in edges[e]:
                edges[e].append(hub)
    edges.append(list(range(100, 3100)))                       # one 3000-pin hyperedge
    edges = [sorted(int(x) for x in e) for e in edges]
    eptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    pins = np.array([p for e in edges for p in e], dtype=np.int32)
    w = np.concatenate([h.w, [1.5]]).astype(np.float32)
    return Hypergraph(n=h.n, m=len(edges), eptr=eptr, pins=pins, w=w)


def test_rating_from_the_librarys_resistances():
    h = _with_hubs(generate(12000, 12500, 2, 400, 2.7828, p_loc=0.7, weights="lognormal",
                            seed=21), 22)
    say(f"case: hef_rating n={h.n} m={h.m} nnz={h.nnz} max|e|={h.sizes().max()} "
        f"max degree {np.bincount(h.pins, minlength=h.n).max()}")
    R, _, _ = hef.resistance(to_device(h), hef.Params(k=10, b=4))
    R = R.cpu().numpy()
    _check(h, R, 0.0)
    _check(h, R, 1.0)


def test_rating_is_equation_7_for_cardinality_resistances():
    h = generate(3000, 3200, 2, 30, 2.5, p_loc=0.5, win=200, weights="lognormal", seed=23)
    say("case: hef_rating with R_e = |e| and shift 1 (Eq. (7))")
    _check(h, np.diff(h.eptr).astype(np.float32), 1.0)


def test_rating_in_several_batches():
    """More triples than one batch holds (at least 2^20): the nodes are
    rated batch by batch."""
    h = generate(30000, 30000, 2, 2000, 2.4, p_loc=0.7, win=500, weights="lognormal", seed=24)
    tri = int((np.diff(h.eptr) * (np.diff(h.eptr) - 1)).sum())
    say(f"case: hef_rating batched: {tri} triples, nnz {h.nnz}")
    assert tri > 2 * max(h.nnz, 1 << 20)
    R = np.random.default_rng(25).random(h.m).astype(np.float32) + 0.01
    nodes = np.random.default_rng(26).choice(h.n, size=400, replace=False)
    _check(h, R, 0.0, nodes)


def test_rating_errors_and_degenerate_cases():
    h = generate(500, 520, 2, 8, 2.5, seed=27)
    dh = to_device(h)
    R = torch.rand(h.m, device="cuda")
    R[3] = float("nan")
    say("case: hef_rating with a non-finite resistance")
    with pytest.raises(hef.HefError) as ei:
        hef.rating(dh, R, 0.0)
    assert ei.value.status == 1
    # R_e equal to the shift: the hyperedge adds nothing (and its pins still
    # count as neighbours)
    R = np.full(h.m, 0.5, np.float32)
    R[::3] = 1.0
    say("case: hef_rating with zero denominators")
    _check(h, R, 1.0)
