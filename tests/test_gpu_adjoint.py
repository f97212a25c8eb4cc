"""GPU parity of the adjoint (dL/dw for L = sum_e c_e R_e) through the C ABI.

* against the float64 autograd gradient of the oracle (same seeded inputs):
  within 1e-3 norm-relative (the FP32 forward error of about 1e-5,
  amplified by the conditioning of the Krylov recurrence, with a margin), on
  hyperedges whose selected branch (largest ratio column,
  largest / smallest pin) is the same on both sides;
* Euler's identity: R is homogeneous of degree -1 in w, so w . dL/dw = -L;
* at the full gradient workload (200k nodes, 210k hyperedges, lognormal
  weights, k = 20, b = 4): the oracle gradient, Euler's identity and bitwise
  determinism; independence of the checkpoint interval (bitwise).
"""
import os

import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from oracle import gradient as ogr
from synth import generate, get_config, make_hypergraph
from tests.gpu_common import say, starts, to_device

pytestmark = pytest.mark.gpu


def _gpu_grad(h, k, b, coef, **kw):
    dh = to_device(h)
    Xs, Xc, xs, xc = starts(h, b)
    p = hef.Params(k=k, b=b, **kw)
    R, _, _ = hef.resistance(dh, p, xs, xc)
    dR = torch.as_tensor(coef.astype(np.float32), device="cuda")
    dw = hef.resistance_backward(dh, p, dR, xs, xc)
    return Xs, Xc, R.cpu().numpy().astype(np.float64), dw.cpu().numpy().astype(np.float64)


def _branch_agrees(R_gpu, R_ref):
    # hyperedges whose resistance agrees to 1e-5 (the same branch is taken)
    return np.abs(R_gpu - R_ref) <= 1e-5 * np.maximum(np.abs(R_ref), 1e-12)


CASES = [
    # (n, m, size range, alpha, locality, window, b, k, seed)
    (300, 320, (2, 12), 2.5, 0.5, 100, 2, 5, 4),
    (2000, 2100, (2, 20), 2.5, 0.5, 200, 1, 10, 8),
    (6000, 6400, (2, 300), 2.2, 0.7, 400, 4, 8, 31),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}_b{c[6]}_k{c[7]}")
def test_gradient_matches_oracle(case):
    n, m, (lo, hi), alpha, ploc, win, b, k, seed = case
    h = generate(n, m, lo, hi, alpha, p_loc=ploc, win=win, weights="lognormal", seed=seed)
    coef = np.random.default_rng(seed + 100).standard_normal(h.m)
    say(f"case: adjoint vs oracle n={h.n} m={h.m} b={b} k={k} max|e|={h.sizes().max()}")
    Xs, Xc, R, dw = _gpu_grad(h, k, b, coef)
    L_ref, g_ref, R_ref = ogr.loss_and_grad(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k, coef)
    err = np.linalg.norm(dw - g_ref) / np.linalg.norm(g_ref)
    same = _branch_agrees(R, R_ref)
    say(f"  dw norm-rel err {err:.2e}; R agree on {same.mean():.4f} of hyperedges")
    assert err < 1e-3
    L = float(coef @ R)
    euler = float(h.w.astype(np.float64) @ dw)
    say(f"  Euler: w.dw = {euler:.6e}, -L = {-L:.6e}")
    assert abs(euler + L) <= 1e-3 * abs(L)


def test_checkpoint_interval_and_determinism():
    h = generate(3000, 3200, 2, 40, 2.5, p_loc=0.6, win=200, weights="lognormal", seed=17)
    coef = np.random.default_rng(3).standard_normal(h.m)
    dh = to_device(h)
    dR = torch.as_tensor(coef.astype(np.float32), device="cuda")
    outs = []
    for ck in (0, 1, 3, 7, 5, 5):
        say(f"case: adjoint ckpt_every={ck} n={h.n} k=12 b=2")
        outs.append(hef.resistance_backward(dh, hef.Params(k=12, b=2, ckpt_every=ck), dR))
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("flags", ["star_only", "clique_only"])
def test_single_expansion_euler(flags):
    h = generate(2000, 2100, 2, 20, 2.5, p_loc=0.5, win=200, weights="lognormal", seed=9)
    coef = np.random.default_rng(5).standard_normal(h.m)
    say(f"case: adjoint {flags} n={h.n} k=10 b=2")
    kw = {flags: True}
    dh = to_device(h)
    p = hef.Params(k=10, b=2, **kw)
    R, _, _ = hef.resistance(dh, p)
    dw = hef.resistance_backward(dh, p, torch.as_tensor(coef.astype(np.float32), device="cuda"))
    L = float(coef @ R.cpu().numpy().astype(np.float64))
    euler = float(h.w.astype(np.float64) @ dw.cpu().numpy().astype(np.float64))
    say(f"  Euler: w.dw = {euler:.6e}, -L = {-L:.6e}")
    assert np.isfinite(dw.cpu().numpy()).all()
    assert abs(euler + L) <= 1e-3 * abs(L)


def test_taped_forward_matches_forward_and_backward():
    h = generate(3000, 3200, 2, 40, 2.5, p_loc=0.6, win=200, weights="lognormal", seed=23)
    dh = to_device(h)
    p = hef.Params(k=10, b=2)
    say(f"case: taped forward n={h.n}")
    R0, _, _ = hef.resistance(dh, p)
    R1, tape = hef.resistance_taped(dh, p)
    assert torch.equal(R0, R1)
    dR = torch.randn(h.m, device="cuda", generator=torch.Generator("cuda").manual_seed(4))
    g_tape = hef.resistance_backward(dh, p, dR, tape=tape)
    g_full = hef.resistance_backward(dh, p, dR)
    assert torch.equal(g_tape, g_full)


def test_autograd_function():
    h = generate(1000, 1100, 2, 15, 2.5, p_loc=0.5, win=100, weights="lognormal", seed=21)
    dh = to_device(h)
    p = hef.Params(k=6, b=2)
    w = dh.w.clone().requires_grad_(True)
    say(f"case: HyperEFResistance autograd n={h.n}")
    R = hef.HyperEFResistance.apply(w, dh, p)
    coef = torch.randn(h.m, device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    (coef * R).sum().backward()
    direct = hef.resistance_backward(dh, p, coef)
    assert torch.equal(w.grad, direct)


def test_full_size_gradient_matches_oracle():
    """The gradient workload at its full size against the float64 autograd
    oracle on the same start blocks, stored by a script that calls only the
    oracle (it takes minutes on the CPU).  A dense finite difference of the
    FP32 forward is no check here: with 160 columns a relative perturbation
    of every weight moves many hyperedges across a switch of their largest
    ratio, where R has a kink."""
    cfg = get_config("grad200k")
    h = make_hypergraph("grad200k")
    k, b = cfg["k"], cfg["b"]
    say(f"case: adjoint grad200k n={h.n} m={h.m} k={k} b={b}")
    coef = np.random.default_rng(7).standard_normal(h.m)
    Xs, Xc, R, dw = _gpu_grad(h, k, b, coef)
    dh = to_device(h)
    _, _, xs, xc = starts(h, b)
    dw2 = hef.resistance_backward(dh, hef.Params(k=k, b=b),
                                  torch.as_tensor(coef.astype(np.float32), device="cuda"), xs, xc)
    assert np.array_equal(dw2.cpu().numpy().astype(np.float64), dw)
    assert np.isfinite(dw).all()
    w0 = h.w.astype(np.float64)
    L = float(coef @ R)
    say(f"  Euler: w.dw = {w0 @ dw:.6e}, -L = {-L:.6e}")
    assert abs(w0 @ dw + L) <= 1e-3 * abs(L)
    # written by tests/golden/make_grad200k.py (oracle only, same inputs)
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "grad200k_dw.npz"))
    g_ref = ref["dw"].astype(np.float64)
    err = np.linalg.norm(dw - g_ref) / np.linalg.norm(g_ref)
    say(f"  L gpu {L:.9e} oracle {float(ref['L']):.9e}; dw norm-rel err vs oracle {err:.2e}")
    assert abs(L - float(ref["L"])) <= 1e-4 * abs(float(ref["L"]))
    assert err < 1e-3
    # central differences of the float64 forward on 64 weights (written by
    # tests/golden/make_grad200k_fd.py, oracle only): the same statistics
    # as the oracle gradient meets, with the FP32 path's own error on top
    fd = np.load(os.path.join(os.path.dirname(__file__), "golden", "grad200k_fd.npz"))
    idx, q, cs = fd["idx"], fd["fd"], fd["column_switches"]
    g_idx = dw[idx]
    rel = np.abs(q - g_idx) / np.abs(g_idx)
    quiet = cs == 0
    say(f"  vs FD on {len(idx)} weights: median rel {np.median(rel):.2e}, "
        f"within 2e-2 {(rel <= 2e-2).mean():.2f}, quiet {quiet.sum()}")
    assert np.linalg.norm((q - g_idx)[quiet]) <= 2e-3 * np.linalg.norm(g_idx[quiet])
    assert np.median(rel) <= 2e-3
    assert (rel <= 2e-2).mean() >= 0.9
    assert np.corrcoef(q, g_idx)[0, 1] >= 0.999


def test_wide_pool_with_more_than_2_31_score_entries():
    """m x K above 2^31 (4.25M hyperedges, K = 512): the score adjoint's
    per-(e, i) slices and the forward's stored numerators sit past 2^31
    entries of the workspace.  Euler's identity w . dL/dw = -L (R is
    homogeneous of degree -1 in w) holds at any size; c_e > 0 keeps L free of
    cancellation."""
    n, m = 1_000_000, 4_250_000
    h = generate(n, m, 2, 6, 2.5, p_loc=0.7, win=200, weights="lognormal", seed=77)
    p = hef.Params(k=32, b=16, star_only=True, assume_valid=True)
    K = p.K
    say(f"case: wide pool n={h.n} m={h.m} nnz={h.nnz} K={K} m*K={h.m * K} (2^31={2**31})")
    assert h.m * K > 2 ** 31
    dh = to_device(h)
    coef = 1.0 + 0.5 * np.random.default_rng(78).random(h.m)
    R, _, _ = hef.resistance(dh, p)
    dw = hef.resistance_backward(dh, p, torch.as_tensor(coef.astype(np.float32), device="cuda"))
    R = R.cpu().numpy().astype(np.float64)
    dw = dw.cpu().numpy().astype(np.float64)
    L = float(coef @ R)
    euler = float(h.w.astype(np.float64) @ dw)
    say(f"  L={L:.6e} w.dw={euler:.6e} rel {abs(euler + L) / abs(L):.2e}")
    assert np.isfinite(R).all() and np.isfinite(dw).all() and (R >= 0).all()
    assert abs(euler + L) <= 1e-3 * abs(L)
