"""Pins of the FP64 oracle for Alg. 1 against what the paper and mathematics fix.

Every check here is independent of the oracle's own formulas: dense builds
from the expansion definitions, spectral facts of normalised adjacencies,
high-precision Gram-Schmidt of the power basis, brute force over pin pairs,
exact identities of Eqs. (9) and (13), pseudo-inverse bounds from Eq. (6) and
the convex program of Eq. (8).
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import exact
from oracle import resistance as orr
from synth import generate, make_hypergraph, start_block
from synth.configs import graph_2uniform


def _small(seed=3, n=40, m=45, weights="lognormal"):
    return generate(n, m, 2, 8, 2.5, weights=weights, seed=seed)


def _est(h, k=10, b=1, seed=7, **kw):
    Xs = start_block(seed, 0, 0, h.n + h.m, b)
    Xc = start_block(seed, 0, 1, h.n, b)
    return orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k, **kw)


# ---------------------------------------------------------------- operators

@pytest.mark.parametrize("seed", [1, 2])
def test_sparse_expansions_equal_dense_definitions(seed):
    h = _small(seed)
    args = (h.n, h.m, h.eptr, h.pins, h.w)
    assert np.allclose(orr.star_weights(*args).toarray(), orr.dense_star_weights(*args), atol=1e-15)
    assert np.allclose(orr.clique_weights(*args).toarray(), orr.dense_clique_weights(*args), atol=1e-15)


def test_clique_degree_is_twice_star_degree():
    h = _small(5)
    args = (h.n, h.m, h.eptr, h.pins, h.w)
    db = np.asarray(orr.star_weights(*args).sum(1)).ravel()[:h.n]
    dc = np.asarray(orr.clique_weights(*args).sum(1)).ravel()
    assert np.allclose(dc, 2 * db, rtol=1e-14)
    # and a star hyperedge-node degree is w_e (d(e) read as |e|)
    de = np.asarray(orr.star_weights(*args).sum(1)).ravel()[h.n:]
    assert np.allclose(de, h.w, rtol=1e-6)


def test_normalised_adjacency_spectral_facts():
    h = _small(7)
    args = (h.n, h.m, h.eptr, h.pins, h.w)
    for W in (orr.star_weights(*args), orr.clique_weights(*args)):
        A = orr.normalized_adjacency(W)
        d = np.asarray(W.sum(1)).ravel()
        v = np.sqrt(d)
        assert np.allclose(A @ v, v, atol=1e-12)               # eigenvalue 1
        assert abs(A - A.T).max() < 1e-15                      # symmetric
        ev = np.linalg.eigvalsh(A.toarray())
        assert ev.max() < 1 + 1e-12 and ev.min() > -1 - 1e-12  # spectrum in [-1, 1]
    # star expansion is bipartite: the sign-flipped vector has eigenvalue -1
    W = orr.star_weights(*args)
    A = orr.normalized_adjacency(W)
    v = np.sqrt(np.asarray(W.sum(1)).ravel())
    v[h.n:] *= -1
    assert np.allclose(A @ v, -v, atol=1e-12)


def test_operators_invariant_to_weight_scale():
    h = _small(9)
    for f in (orr.star_operator, orr.clique_operator):
        A1 = f(h.n, h.m, h.eptr, h.pins, h.w)
        A2 = f(h.n, h.m, h.eptr, h.pins, 3.0 * h.w.astype(np.float64))
        assert abs(A1 - A2).max() < 1e-14


# ------------------------------------------------------------------- pool

def _mp_gs(M, digits=60):
    """Classical Gram-Schmidt in `digits`-digit arithmetic (mpmath)."""
    mpmath.mp.dps = digits
    A = mpmath.matrix(M.tolist())
    rows, cols = A.rows, A.cols
    Q = mpmath.matrix(rows, cols)
    for j in range(cols):
        v = A[:, j]
        for i in range(j):
            v = v - (Q[:, i].T * A[:, j])[0] * Q[:, i]
        v = v / mpmath.norm(v)
        Q[:, j] = v
    return np.array([[float(Q[r, c]) for c in range(cols)] for r in range(rows)])


def test_pool_matches_high_precision_gram_schmidt_of_power_basis():
    """Each expansion's pool vector q_j equals (up to sign) the j-th vector of
    a 60-digit Gram-Schmidt of [x, Ax, ..., A^k x], with x dropped; then the
    joint pool equals the 60-digit Gram-Schmidt of [star node parts | clique]."""
    h = make_hypergraph("pinv50")
    k = 6
    Xs = start_block(7, 0, 0, h.n + h.m, 1)
    Xc = start_block(7, 0, 1, h.n, 1)
    est = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k)
    assert est.pool.chi.shape[1] == 2 * k
    cols = []
    for A, X, blocks in ((orr.star_operator(h.n, h.m, h.eptr, h.pins, h.w), Xs, est.pool.star_blocks),
                         (orr.clique_operator(h.n, h.m, h.eptr, h.pins, h.w), Xc, est.pool.clique_blocks)):
        A = A.toarray()
        mpmath.mp.dps = 60
        Am = mpmath.matrix(A.tolist())
        v = mpmath.matrix(X.tolist())
        power = [v]
        for _ in range(k):
            v = Am * v
            power.append(v)
        P = np.array([[float(power[j][r]) for j in range(k + 1)] for r in range(A.shape[0])])
        # Gram-Schmidt in high precision directly on the mp vectors
        Q = []
        for j in range(k + 1):
            u = power[j]
            for q in Q:
                u = u - (q.T * power[j])[0] * q
            u = u / mpmath.norm(u)
            Q.append(u)
        Qn = np.array([[float(Q[j][r]) for j in range(k + 1)] for r in range(A.shape[0])])
        for j in range(1, k + 1):
            o = blocks[j][:, 0]
            assert min(np.abs(o - Qn[:, j]).max(), np.abs(o + Qn[:, j]).max()) < 1e-9
        cols.append(Qn[:h.n, 1:] if A.shape[0] > h.n else Qn[:, 1:])
        assert P.shape[1] == k + 1
    joint = _mp_gs(np.hstack(cols))
    for j in range(joint.shape[1]):
        o = est.pool.chi[:, j]
        assert min(np.abs(o - joint[:, j]).max(), np.abs(o + joint[:, j]).max()) < 1e-9


def _mp_power_gs(A, X, k, digits=60):
    """60-digit Gram-Schmidt of the step-major power basis
    [x_1 .. x_b, A x_1 .. A x_b, ..., A^k x_1 .. A^k x_b] (float64 out)."""
    mpmath.mp.dps = digits
    Am = mpmath.matrix(A.tolist())
    b = X.shape[1]
    cur = [mpmath.matrix(X[:, c].tolist()) for c in range(b)]
    power = []
    for _ in range(k + 1):
        power += cur
        cur = [Am * v for v in cur]
    Q = []
    for u0 in power:
        u = u0
        for q in Q:
            u = u - (q.T * u0)[0] * q
        Q.append(u / mpmath.norm(u))
    return np.array([[float(q[r]) for q in Q] for r in range(A.shape[0])])


def test_block_pool_matches_high_precision_gram_schmidt_step_major():
    """b = 2: column c of Krylov block j equals column j*b + c of the 60-digit
    Gram-Schmidt of the step-major power basis (start vectors of one step
    first, then their images), for both expansions; the joint pool is then
    the 60-digit Gram-Schmidt of [star node parts | clique], each part in
    step-major order.  A block laid out expansion-major or column-major
    (x_1, A x_1, ..., x_2, A x_2, ...) fails this."""
    h = make_hypergraph("pinv50")
    k, b = 4, 2
    Xs = start_block(7, 0, 0, h.n + h.m, b)
    Xc = start_block(7, 0, 1, h.n, b)
    est = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k)
    assert est.pool.chi.shape[1] == 2 * b * k
    cols = []
    for A, X, blocks, rows in ((orr.star_operator(h.n, h.m, h.eptr, h.pins, h.w), Xs,
                                est.pool.star_blocks, h.n),
                               (orr.clique_operator(h.n, h.m, h.eptr, h.pins, h.w), Xc,
                                est.pool.clique_blocks, h.n)):
        Qn = _mp_power_gs(A.toarray(), X, k)
        assert len(blocks) == k + 1
        for j in range(k + 1):
            assert blocks[j].shape[1] == b
            for c in range(b):
                o, ref = blocks[j][:, c], Qn[:, j * b + c]
                assert min(np.abs(o - ref).max(), np.abs(o + ref).max()) < 1e-9, (j, c)
        cols.append(Qn[:rows, b:])
    joint = _mp_gs(np.hstack(cols))
    for j in range(joint.shape[1]):
        o = est.pool.chi[:, j]
        assert min(np.abs(o - joint[:, j]).max(), np.abs(o + joint[:, j]).max()) < 1e-9, j


def test_fullsize_golden_script_equals_the_oracle():
    """The script that writes the full-size oracle samples computes exactly
    orr.resistance (it only frees each expansion's blocks early)."""
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "make_fullsize_samples.py")
    spec = importlib.util.spec_from_file_location("make_fullsize_samples", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    h = make_hypergraph("tiny2k")
    Xs = start_block(7, 0, 0, h.n + h.m, 2)
    Xc = start_block(7, 0, 1, h.n, 2)
    R, qh = mod.lean_resistance(h, Xs, Xc, 5)
    ref = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, 5)
    assert np.array_equal(R, ref.R) and np.array_equal(qh, ref.qh)


def test_pool_orthonormal_and_well_conditioned():
    h = make_hypergraph("tiny2k")
    est = _est(h, k=10, b=1)
    chi = est.pool.chi
    assert chi.shape == (h.n, 20)
    assert np.abs(chi.T @ chi - np.eye(20)).max() < 1e-13
    assert est.pool.rho.min() > 0.5
    # Krylov blocks of each expansion are mutually orthonormal in their own space
    B = np.hstack(est.pool.star_blocks)
    assert np.abs(B.T @ B - np.eye(B.shape[1])).max() < 1e-13


def test_rank_deficient_pool_drops_columns():
    """A hypergraph with a single hyperedge has a 2-dimensional star space
    beyond the pins' common value: the Krylov sequence breaks down and the
    drop rule removes the dependent columns."""
    n = 3
    eptr = np.array([0, 3])
    pins = np.array([0, 1, 2])
    w = np.array([2.0], dtype=np.float32)
    Xs = start_block(1, 0, 0, n + 1, 1)
    Xc = start_block(1, 0, 1, n, 1)
    est = orr.resistance(n, 1, eptr, pins, w, Xs, Xc, 5)
    assert est.pool.chi.shape[1] <= n
    chi = est.pool.chi
    assert np.abs(chi.T @ chi - np.eye(chi.shape[1])).max() < 1e-12


# ----------------------------------------------------------------- scores

def test_spread_equals_brute_force_pair_maximum():
    h = _small(11)
    rng = np.random.default_rng(0)
    chi = rng.standard_normal((h.n, 5))
    s = orr.edge_spread(h.eptr, h.pins, chi)
    for e in range(h.m):
        mem = chi[h.pins[h.eptr[e]:h.eptr[e + 1]]]
        brute = ((mem[:, None, :] - mem[None, :, :]) ** 2).max(axis=(0, 1))
        assert np.allclose(s[e], brute, rtol=1e-15, atol=0)


def test_quadratic_form_equals_eq9_brute_force():
    h = _small(12)
    chi = np.random.default_rng(1).standard_normal((h.n, 3))
    qh = orr.quadratic_forms(h.eptr, h.pins, h.w, chi)
    for i in range(3):
        assert math.isclose(qh[i], exact.q_h(h.eptr, h.pins, h.w, chi[:, i]), rel_tol=1e-13)


def test_weighted_ratios_sum_to_one():
    """Eq. (13) with Eq. (9): sum_e w_e r_e(chi) = Q_H(chi)/Q_H(chi) = 1."""
    h = make_hypergraph("tiny2k")
    est = _est(h)
    s = orr.edge_spread(h.eptr, h.pins, est.pool.chi)
    tot = (h.w.astype(np.float64)[:, None] * s / est.qh[None, :]).sum(0)
    assert np.abs(tot - 1).max() < 1e-13


def test_single_hyperedge_resistance_is_inverse_weight():
    for size, wv in ((2, 1.0), (5, 0.25), (9, 3.0)):
        n = size + 2
        eptr = np.array([0, size])
        pins = np.arange(1, size + 1)
        w = np.array([wv], dtype=np.float32)
        Xs = start_block(3, 0, 0, n + 1, 1)
        Xc = start_block(3, 0, 1, n, 1)
        est = orr.resistance(n, 1, eptr, pins, w, Xs, Xc, 3)
        assert math.isclose(est.R[0], 1.0 / wv, rel_tol=1e-12)


def test_resistance_bounded_by_inverse_weight():
    h = _small(13, n=200, m=220)
    est = _est(h, k=8, b=2)
    assert (est.R <= 1.0 / h.w.astype(np.float64) * (1 + 1e-12)).all()
    assert (est.R >= 0).all()


def test_pseudo_inverse_bounds():
    """Q_H >= chi^T L_c chi and Q_H >= 4 chi^T S_b chi (S_b: star Laplacian
    reduced to V), so R_e <= max_{p,q in e} R_eff^{G_c}(p,q) and
    R_e <= max R_eff^{G_b}(p,q) / 4 (Eq. (6))."""
    h = make_hypergraph("pinv50")
    est = _est(h)
    args = (h.n, h.m, h.eptr, h.pins, h.w)
    Rc = exact.max_pair(exact.pinv_resistance(orr.dense_clique_weights(*args)), h.eptr, h.pins)
    Rb = exact.max_pair(exact.pinv_resistance(orr.dense_star_weights(*args)), h.eptr, h.pins)
    conn = np.isfinite(Rc) & (Rc < 1e8)
    assert (est.R[conn] <= Rc[conn] * (1 + 1e-9)).all()
    assert (est.R[conn] <= Rb[conn] / 4 * (1 + 1e-9)).all()
    assert est.R.max() > 0


def test_two_uniform_hypergraph_is_bounded_by_graph_resistance():
    """For a simple graph Q_H(chi) = chi^T L chi, so each ratio is a lower
    bound of R_eff(p, q) = b_pq^T L^+ b_pq (Eq. (6))."""
    g = graph_2uniform(50, 120)
    est = _est(g)
    W = np.zeros((g.n, g.n))
    for e in range(g.m):
        p, q = g.pins[2 * e], g.pins[2 * e + 1]
        W[p, q] += g.w[e]
        W[q, p] += g.w[e]
    Reff = exact.pinv_resistance(W)
    for e in range(g.m):
        p, q = g.pins[2 * e], g.pins[2 * e + 1]
        assert est.R[e] <= Reff[p, q] * (1 + 1e-9)
        chi = est.pool.chi
        lap = chi.T @ exact.laplacian(W) @ chi
        assert np.allclose(np.diag(lap), est.qh, rtol=1e-10)


def test_estimate_below_exact_resistance_diameter():
    """R_e restricts the maximisation of Eq. (8) to the pool columns, so it
    never exceeds R*_e (solved as a convex program on a 7-node hypergraph)."""
    n = 7
    eptr = np.array([0, 3, 5, 7, 10, 12])
    pins = np.array([0, 1, 2, 2, 3, 3, 4, 4, 5, 6, 0, 6])
    w = np.array([1.0, 2.0, 0.5, 1.5, 1.0], dtype=np.float32)
    Xs = start_block(5, 0, 0, n + 5, 1)
    Xc = start_block(5, 0, 1, n, 1)
    est = orr.resistance(n, 5, eptr, pins, w, Xs, Xc, 4)
    for e in range(5):
        Rstar = exact.exact_resistance_diameter(n, eptr, pins, w, e)
        assert est.R[e] <= Rstar * (1 + 1e-6)
        assert Rstar <= 1.0 / w[e] * (1 + 1e-6)


def test_homogeneity_in_weights():
    h = _small(14, n=100, m=110)
    Xs = start_block(7, 0, 0, h.n + h.m, 2)
    Xc = start_block(7, 0, 1, h.n, 2)
    R1 = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, 6).R
    for c in (0.5, 3.0):
        Rc = orr.resistance(h.n, h.m, h.eptr, h.pins, c * h.w.astype(np.float64), Xs, Xc, 6).R
        assert np.allclose(Rc, R1 / c, rtol=1e-10)


def test_mixed_pool_dominates_star_only():
    h = make_hypergraph("tiny2k")
    Rm = _est(h).R
    Rs = _est(h, use_clique=False).R
    assert (Rm >= Rs * (1 - 1e-10)).all()
    assert Rm.mean() > Rs.mean()


def test_permutation_equivariance():
    h = _small(15, n=120, m=130)
    b, k = 2, 6
    Xs = start_block(7, 0, 0, h.n + h.m, b)
    Xc = start_block(7, 0, 1, h.n, b)
    R = orr.resistance(h.n, h.m, h.eptr, h.pins, h.w, Xs, Xc, k).R
    rng = np.random.default_rng(2)
    pn = rng.permutation(h.n)          # new id of node v is pn[v]
    pe = rng.permutation(h.m)          # new hyperedge i is old pe[i]
    eptr, pins = [0], []
    for e in pe:
        mem = np.sort(pn[h.pins[h.eptr[e]:h.eptr[e + 1]]])
        pins.extend(mem.tolist())
        eptr.append(len(pins))
    inv = np.argsort(pn)
    Xs2 = np.vstack([Xs[:h.n][inv], Xs[h.n:][pe]])
    Xc2 = Xc[inv]
    R2 = orr.resistance(h.n, h.m, np.array(eptr), np.array(pins), h.w[pe], Xs2, Xc2, k).R
    assert np.allclose(R2, R[pe], rtol=1e-9, atol=1e-15)
