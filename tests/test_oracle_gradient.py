"""Pins of the oracle gradient of L(w) = sum_e c_e R_e(w).

* the torch forward equals the NumPy oracle forward (same definitions);
* central finite differences of the NumPy oracle (h = 1e-4) agree with the
  autograd gradient on coordinates where no maximum switches branch;
* Euler's identity: R is homogeneous of degree -1 in w (the normalised
  adjacencies do not change under w -> c w, Q_H scales by c), so
  w . grad L = -L exactly.
"""
import numpy as np

from oracle import gradient as ogr
from oracle import resistance as orr
from synth import generate, start_block


def _case(seed=4, n=300, m=320, b=2, k=5):
    h = generate(n, m, 2, 12, 2.5, p_loc=0.5, win=100, weights="lognormal", seed=seed)
    Xs = start_block(7, 0, 0, h.n + h.m, b)
    Xc = start_block(7, 0, 1, h.n, b)
    coef = np.random.default_rng(11).standard_normal(h.m)
    return h, Xs, Xc, k, coef


def test_torch_forward_equals_numpy_oracle():
    h, Xs, Xc, k, coef = _case()
    L, g, R = ogr.loss_and_grad(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k, coef)
    Ro = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k).R
    assert np.allclose(R, Ro, rtol=1e-9, atol=1e-15)
    assert np.isclose(L, (coef * Ro).sum(), rtol=1e-9)


def test_euler_identity():
    h, Xs, Xc, k, coef = _case(5)
    L, g, _ = ogr.loss_and_grad(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k, coef)
    assert np.isclose(float(h.w.astype(np.float64) @ g), -L, rtol=1e-9)


def test_central_differences():
    h, Xs, Xc, k, coef = _case(6, n=150, m=160, k=4)
    w0 = h.w.astype(np.float64)
    L, g, _ = ogr.loss_and_grad(h.n, h.m, h.eptr, h.pins, w0, Xs, Xc, k, coef)
    rng = np.random.default_rng(13)
    idx = rng.choice(h.m, size=24, replace=False)
    step = 1e-4

    def forward(w):
        est = orr.resistance(h.n, h.m, h.eptr, h.pins, w, Xs, Xc, k)
        s = orr.edge_spread(h.eptr, h.pins, est.pool.chi)
        # every branch the maxima take: best column, largest and smallest pin
        G = est.pool.chi[h.pins]
        hi = np.stack([G[h.eptr[e]:h.eptr[e + 1]].argmax(0) for e in range(h.m)])
        lo = np.stack([G[h.eptr[e]:h.eptr[e + 1]].argmin(0) for e in range(h.m)])
        return (coef * est.R).sum(), np.concatenate([(s / est.qh).argmax(1)[:, None], hi, lo], 1)

    _, arg0 = forward(w0)
    checked = 0
    for i in idx:
        wp, wm = w0.copy(), w0.copy()
        wp[i] += step
        wm[i] -= step
        Lp, ap = forward(wp)
        Lm, am = forward(wm)
        if not (np.array_equal(ap, arg0) and np.array_equal(am, arg0)):
            continue                      # a maximum switched branch: skip
        fd = (Lp - Lm) / (2 * step)
        assert abs(fd - g[i]) <= 1e-5 * max(abs(g).max(), 1e-12) + 1e-4 * abs(g[i]), (i, fd, g[i])
        checked += 1
    assert checked >= 12


def test_fullsize_gradient_matches_central_differences():
    """The gradient workload at its full size (200k nodes, 210k hyperedges,
    k = 20, b = 4): the stored float64 autograd gradient against central
    differences of the float64 forward on 64 weights, both written by
    scripts under tests/golden/ that call only the oracle.  At this size some
    maximum somewhere always changes branch inside +-h (a kink of R, whose
    one-sided slopes differ); the stored switch counts say how many.  Where
    no hyperedge's ratio column switches, the quotient is the derivative up
    to the pin-level kinks: agreement to 1e-3; everywhere, the median
    relative error and the spread are those of a derivative."""
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    fd = np.load(os.path.join(here, "grad200k_fd.npz"))
    g = np.load(os.path.join(here, "grad200k_dw.npz"))
    idx, q, cs = fd["idx"], fd["fd"], fd["column_switches"]
    dw = g["dw"].astype(np.float64)[idx]
    rel = np.abs(q - dw) / np.abs(dw)
    quiet = cs == 0
    assert quiet.sum() >= 4
    assert np.linalg.norm((q - dw)[quiet]) <= 1e-3 * np.linalg.norm(dw[quiet])
    assert np.median(rel) <= 1e-3
    assert (rel <= 2e-2).mean() >= 0.9
    assert np.corrcoef(q, dw)[0, 1] >= 0.9999
