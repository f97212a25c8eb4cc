"""GPU parity of Alg. 1 (a1-a5): the HIP path against the FP64 oracle on the
same seeded inputs, through the C ABI.

Tolerances: FP32 R within 1e-4 norm-relative and 1e-4 at the 99.9th
percentile of elementwise relative error over hyperedges with R >= 1e-3 max R
(FP32 rounding through k Krylov steps and the joint orthonormalisation,
measured at about 1e-6 to 1e-5); Q_H within 1e-5 relative; the BF16 pool
within 1e-2 norm-relative (bf16 rounding is 2^-9 relative per element).
"""
import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from oracle import resistance as orr
from synth import generate, make_hypergraph, start_block
from tests.gpu_common import r_errors, say, starts, to_device

pytestmark = pytest.mark.gpu


def test_start_block_generator_matches_counter_definition():
    say("case: start_block seed=7 level=2 expansion=1 rows=5000 b=8")
    g = hef.start_block(7, 2, 1, 5000, 8).cpu().numpy()
    ref = start_block(7, 2, 1, 5000, 8)
    assert np.abs(g - ref.astype(np.float32)).max() <= 1e-6 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("b", [1, 4, 8, 16])
def test_expansion_operators_match_oracle(b):
    # hyperedges up to 300 pins exercise the long-segment CSR kernel (csr_big);
    # node degrees stay below 32 here: test_long_node_segments covers csc_big
    h = generate(6000, 6400, 2, 300, 2.2, p_loc=0.7, win=400, weights="lognormal", seed=31)
    say(f"case: debug_apply n={h.n} m={h.m} b={b} maxsize={h.sizes().max()}")
    dh = to_device(h)
    rng = np.random.default_rng(b)
    for expansion, A in ((0, orr.star_operator(h.n, h.m, h.eptr, h.pins, h.w)),
                         (1, orr.clique_operator(h.n, h.m, h.eptr, h.pins, h.w))):
        x = rng.standard_normal((A.shape[0], b)).astype(np.float32)
        y = hef.debug_apply(dh, expansion, torch.as_tensor(x, device="cuda")).cpu().numpy()
        ref = A @ x.astype(np.float64)
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        say(f"  expansion {expansion}: rel err {err:.2e}")
        assert err < 1e-6


def test_gram_kernel_matches_float64():
    rng = np.random.default_rng(5)
    for rows, cols in ((1000, 20), (70_001, 160), (50_000, 480), (333, 37)):
        say(f"case: debug_gram rows={rows} cols={cols}")
        X = rng.standard_normal((rows, cols)).astype(np.float32)
        G = hef.debug_gram(torch.as_tensor(X, device="cuda")).cpu().numpy()
        ref = X.astype(np.float64).T @ X.astype(np.float64)
        err = np.abs(G - ref).max() / np.abs(ref).max()
        say(f"  max rel err {err:.2e}")
        assert err < 2e-6
        assert np.array_equal(G, G.T)


def _parity(h, k, b, basis="fp32", tol_norm=1e-4, tol_p999=1e-4, tol_qh=1e-5, **kw):
    Xs, Xc, xs, xc = starts(h, b)
    est = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k)
    dh = to_device(h)
    R, qh, chi = hef.resistance(dh, hef.Params(k=k, b=b, basis=basis, **kw), xs, xc,
                                return_pool=True)
    R = R.cpu().numpy()
    qh = qh.cpu().numpy()
    norm, p999, mx = r_errors(R, est.R)
    qerr = np.abs(qh - est.qh).max() / est.qh.max()
    say(f"  R norm-rel {norm:.2e} p99.9 {p999:.2e} max {mx:.2e} | qh rel {qerr:.2e}")
    assert norm <= tol_norm and p999 <= tol_p999
    assert qerr <= tol_qh
    return R, qh, chi, est


def test_tiny_fp32_matches_oracle():
    h = make_hypergraph("tiny2k")
    say(f"case: resistance tiny2k n={h.n} k=10 b=1")
    R, qh, chi, est = _parity(h, 10, 1)
    chi = chi.cpu().numpy().astype(np.float64)
    orth = np.abs(chi.T @ chi - np.eye(chi.shape[1])).max()
    say(f"  pool orthogonality {orth:.1e}")
    assert orth < 1e-5
    # sum_e w_e r_e = 1 for every column of the GPU pool (Eqs. (9), (13))
    s = orr.edge_spread(h.eptr, h.pins, chi)
    tot = (h.w.astype(np.float64)[:, None] * s / qh[None, :]).sum(0)
    assert np.abs(tot - 1).max() < 1e-5
    assert (R >= 0).all() and (R <= 1.0 / h.w * (1 + 1e-5)).all()


@pytest.mark.parametrize("seed", [20251107, 20251108])
def test_tiny_other_seeds(seed):
    h = make_hypergraph("tiny2k", seed=seed)
    say(f"case: resistance tiny2k seed={seed}")
    _parity(h, 10, 1)


def test_netlist_shaped_block_krylov_matches_oracle():
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=5)
    say(f"case: resistance netlist20k k=30 b=8 (K=480), max |e|={h.sizes().max()}")
    _parity(h, 30, 8)


def test_two_orthonormalisation_passes():
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=6)
    say("case: resistance netlist20k k=20 b=4 orth_passes=2")
    _parity(h, 20, 4, orth_passes=2)


def test_single_expansion_pools():
    h = make_hypergraph("tiny2k")
    Xs, Xc, xs, xc = starts(h, 2)
    dh = to_device(h)
    for flag, kw in (("star_only", dict(use_clique=False)), ("clique_only", dict(use_star=False))):
        say(f"case: resistance tiny2k {flag}")
        est = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, 8, **kw)
        R, qh, _ = hef.resistance(dh, hef.Params(k=8, b=2, **{flag: True}), xs, xc)
        norm, p999, _ = r_errors(R.cpu().numpy(), est.R)
        say(f"  norm {norm:.2e} p99.9 {p999:.2e}")
        assert norm < 1e-4 and p999 < 1e-4


def test_bf16_pool_within_1e2():
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=5)
    say("case: resistance netlist20k k=30 b=8 basis=bf16")
    _parity(h, 30, 8, basis="bf16", tol_norm=1e-2, tol_p999=1.0, tol_qh=1e-2)


@pytest.mark.parametrize("name,k,b", [("tiny2k", 10, 1), ("netlist20k", 30, 8)])
def test_fp64_debug_basis(name, k, b):
    # the float64 basis: the pool, the joint orthonormalisation and the
    # ratios in float64 from the float32 Krylov blocks, so the float32
    # recurrence bounds R's error (same 1e-4 bar) while the pool is
    # orthonormal to 1e-10 (one Cholesky QR loses kappa^2 u, kappa <= 1/drop_tol)
    # and sum_e w_e r_e = 1 (Eqs. (9), (13)) holds to 1e-12
    if name == "tiny2k":
        h = make_hypergraph("tiny2k")
    else:
        h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=5)
    say(f"case: resistance {name} k={k} b={b} basis=fp64")
    R, qh, chi, est = _parity(h, k, b, basis="fp64")
    assert chi.dtype == torch.float64
    chi = chi.cpu().numpy()
    kept = qh > 0
    G = chi[:, kept].T @ chi[:, kept]
    orth = np.abs(G - np.eye(G.shape[0])).max()
    s = orr.edge_spread(h.eptr, h.pins, chi[:, kept])
    tot = (h.w.astype(np.float64)[:, None] * s / qh[None, kept]).sum(0)
    say(f"  pool orthogonality {orth:.1e}, max |sum w r - 1| {np.abs(tot - 1).max():.1e}")
    assert orth < 1e-10
    assert np.abs(tot - 1).max() < 1e-12
    assert not chi[:, ~kept].any()
    # the static-scratch entry point gives the same bits
    if name == "tiny2k":
        _, _, xs, xc = starts(h, b)
        R2, qh2, _ = hef.resistance_static(to_device(h), hef.Params(k=k, b=b, basis="fp64"),
                                           xs, xc)
        assert np.array_equal(R2.cpu().numpy(), R) and np.array_equal(qh2.cpu().numpy(), qh)


@pytest.mark.parametrize("k,b,basis", [(29, 4, "fp32"), (29, 8, "fp32"), (29, 8, "fp64")])
def test_pool_width_off_the_tile_grid(k, b, basis):
    # K = 2 k b = 232 = 7 x 32 + 8 or 464 = 14 x 32 + 16: the last Cholesky
    # panel, the last block column of R^-1 and the last Gram / apply tiles
    # are partial
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=5)
    say(f"case: resistance netlist20k k={k} b={b} (K={2 * k * b}) basis={basis}")
    _parity(h, k, b, basis=basis)


def test_long_recurrence_two_passes():
    # k = 61 steps: the pool is ill-conditioned enough that one FP32 Cholesky
    # QR loses orthogonality (3e-4); the second pass restores it, and R then
    # sits at the float64-basis level of the same FP32 recurrence (p99.9
    # 8.5e-5 there, hence the 2e-4 bar; Q_H 1e-5, hence 2e-5)
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=5)
    say("case: resistance netlist20k k=61 b=4 (K=488) orth_passes=2")
    R, qh, chi, est = _parity(h, 61, 4, orth_passes=2, tol_p999=2e-4, tol_qh=2e-5)
    c = chi.cpu().numpy().astype(np.float64)[:, qh > 0]
    orth = np.abs(c.T @ c - np.eye(c.shape[1])).max()
    say(f"  pool orthogonality {orth:.1e}")
    assert orth < 1e-6


def test_counter_generator_start_matches_explicit_start():
    h = make_hypergraph("tiny2k")
    say("case: resistance tiny2k with NULL start blocks")
    dh = to_device(h)
    p = hef.Params(k=10, b=1, seed=7)
    R0, _, _ = hef.resistance(dh, p)
    _, _, xs, xc = starts(h, 1)
    R1, _, _ = hef.resistance(dh, p, xs, xc)
    assert torch.equal(R0, R1)


def test_deterministic():
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=7)
    say("case: determinism netlist20k k=10 b=4")
    dh = to_device(h)
    p = hef.Params(k=10, b=4)
    a = hef.resistance(dh, p, return_pool=True)
    b = hef.resistance(dh, p, return_pool=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_invalid_inputs_are_reported():
    h = make_hypergraph("tiny2k")
    say("case: invalid hypergraph on the device")
    pins = h.pins.copy()
    pins[h.eptr[3]] = pins[h.eptr[3] + 1]      # duplicate pin
    dh = hef.DeviceHypergraph.from_arrays(h.n, h.m, h.eptr, pins, h.w)
    with pytest.raises(hef.HefError) as ei:
        hef.resistance(dh, hef.Params())
    assert ei.value.status == 2
    w = h.w.copy()
    w[10] = -1.0
    dh = hef.DeviceHypergraph.from_arrays(h.n, h.m, h.eptr, h.pins, w)
    with pytest.raises(hef.HefError) as ei:
        hef.resistance(dh, hef.Params())
    assert ei.value.status == 2


def test_degenerate_single_hyperedge():
    say("case: single hyperedge R = 1/w")
    n = 8
    eptr = np.array([0, 5])
    pins = np.array([1, 2, 4, 5, 7])
    dh = hef.DeviceHypergraph.from_arrays(n, 1, eptr, pins, np.array([0.25], np.float32))
    R, qh, _ = hef.resistance(dh, hef.Params(k=3, b=1))
    assert abs(float(R[0]) - 4.0) < 1e-4


@pytest.mark.parametrize("b", [1, 4, 8, 16])
def test_long_node_segments(b):
    """Nodes in hundreds of hyperedges (degree >> 32) go to the CSC pass's
    wave-per-node path: six hub nodes are added as pins to 400-900 random
    hyperedges each."""
    base = generate(5000, 6000, 2, 40, 2.5, p_loc=0.7, win=300, weights="lognormal", seed=71)
    rng = np.random.default_rng(72)
    hubs = np.array([3, 777, 1500, 2501, 3999, 4998])
    edges = [list(base.pins[base.eptr[e]:base.eptr[e + 1]]) for e in range(base.m)]
    for i, hub in enumerate(hubs):
        for e in rng.choice(base.m, size=400 + 100 * i, replace=False):
            if hub not in edges[e]:
                edges[e].append(int(hub))
    edges = [sorted(e) for e in edges]
    eptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    pins = np.array([p for e in edges for p in e], dtype=np.int32)
    from synth.hypergraph import Hypergraph
    h = Hypergraph(n=base.n, m=base.m, eptr=eptr, pins=pins, w=base.w)
    deg = np.bincount(pins, minlength=h.n)
    say(f"case: debug_apply hub nodes b={b}: max degree {deg.max()}, "
        f"{int((deg > 32).sum())} nodes above 32")
    assert (deg > 32).sum() >= 6 and deg.max() > 400
    dh = to_device(h)
    rng = np.random.default_rng(b)
    for expansion, A in ((0, orr.star_operator(h.n, h.m, h.eptr, h.pins, h.w)),
                         (1, orr.clique_operator(h.n, h.m, h.eptr, h.pins, h.w))):
        x = rng.standard_normal((A.shape[0], b)).astype(np.float32)
        y = hef.debug_apply(dh, expansion, torch.as_tensor(x, device="cuda")).cpu().numpy()
        ref = A @ x.astype(np.float64)
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        hub_err = np.abs(y[hubs] - ref[hubs]).max() / np.abs(ref[hubs]).max()
        say(f"  expansion {expansion}: rel err {err:.2e}, hub rows {hub_err:.2e}")
        assert err < 1e-6 and hub_err < 1e-6


def test_stage_timing_mask():
    # hef_timing_stages: with only the spmm_step span selected, one event pair
    # per fused SpMM (k Krylov steps), and no other stage; by default every
    # stage but that span
    h = make_hypergraph("tiny2k")
    dh = to_device(h)
    p = hef.Params(k=10, b=1, assume_valid=True)
    say("case: stage timing mask tiny2k k=10 b=1")
    hef.resistance(dh, p)
    torch.cuda.synchronize()
    hef.timing_read(reset=True)
    try:
        hef.timing_stages(["spmm_step"])
        hef.timing_enable(True)
        hef.resistance(dh, p)
        torch.cuda.synchronize()
        hef.timing_enable(False)
        only = {k: v for k, v in hef.timing_read(reset=True).items() if v[1]}
        hef.timing_stages(None)
        hef.timing_enable(True)
        hef.resistance(dh, p)
        torch.cuda.synchronize()
        hef.timing_enable(False)
        full = {k: v for k, v in hef.timing_read(reset=True).items() if v[1]}
    finally:
        hef.timing_enable(False)
        hef.timing_stages(None)
    assert set(only) == {"spmm_step"} and only["spmm_step"][1] == p.k
    assert "spmm_step" not in full
    assert full["spmm_csr"][1] == p.k and full["spmm_csc"][1] == p.k
    assert only["spmm_step"][0] > 0.0
