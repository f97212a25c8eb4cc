"""Alg. 1 (effective-resistance estimation) in plain float64 NumPy/SciPy.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Passages followed (HyperEF 2.0, Section III-A, "Enhanced Estimation of
Hyperedge Effective Resistances", and Alg. 1):

* star expansion G_b: the bipartite graph on V u E with edge weights
  z_b(e, p) = w(e) / d(e); d(e) is read as |e|;
* clique expansion G_c: every node pair u != v of a hyperedge gets
  w(e) / C(|e|, 2), summed over the hyperedges that hold both;
* A is the normalised adjacency D^-1/2 W D^-1/2 of each expansion (the inverse
  square root of a zero degree is taken as 0);
* Eq. (12): Krylov subspace span(x, Ax, ..., A^rho x) from a random start x;
  here a block of b start vectors per expansion and k steps;
* the unified pool: each expansion's Krylov vectors are orthonormalised by
  Gram-Schmidt in the expansion's own space, the random start block is left
  out of the pool, the star vectors lose their entries on star (hyperedge)
  nodes, and the joint list [star | clique] is orthonormalised again
  (Alg. 1);
* Eq. (13): r_e(chi) = (chi_p - chi_q)^2 / Q_H(chi) with p, q the most
  distant pins of e along chi, i.e. the numerator is (max - min)^2 over e;
* Eq. (9): Q_H(chi) = sum_e w_e max_{u,v in e} (chi_u - chi_v)^2;
* Eq. (14): R_e = max_i r_e(chi^(i)).

Readings of silent points (each a named argument):
* ``tau``: a column whose Gram-Schmidt residual is below tau times its length
  (in the per-expansion recurrence: tau times the length of A q before
  orthogonalisation) is dropped;
* a column with Q_H = 0 takes no part in the maximum, and R_e = 0 if no
  column is usable.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# Expansions (Section III-A, star and clique expansion definitions)
# --------------------------------------------------------------------------

def edge_sizes(eptr: np.ndarray) -> np.ndarray:
    return np.diff(np.asarray(eptr, dtype=np.int64))


def incidence(n: int, m: int, eptr, pins) -> sp.csr_matrix:
    """H with H[e, p] = 1 for every pin p of hyperedge e."""
    eptr = np.asarray(eptr, dtype=np.int64)
    pins = np.asarray(pins, dtype=np.int64)
    return sp.csr_matrix((np.ones(pins.shape[0]), pins, eptr), shape=(m, n))


def star_weights(n, m, eptr, pins, w) -> sp.csr_matrix:
    """Weighted adjacency of G_b: node p and hyperedge-node n+e joined with w_e/|e|."""
    H = incidence(n, m, eptr, pins)
    z = np.asarray(w, dtype=np.float64) / edge_sizes(eptr)
    Z = sp.diags(z) @ H                       # m x n, Z[e, p] = w_e / |e|
    return sp.bmat([[None, Z.T], [Z, None]], format="csr")


def clique_weights(n, m, eptr, pins, w) -> sp.csr_matrix:
    """Weighted adjacency of G_c: z_c(u, v) = sum_{e ∋ u,v} w_e / C(|e|, 2), u != v."""
    H = incidence(n, m, eptr, pins)
    s = edge_sizes(eptr).astype(np.float64)
    pair = np.asarray(w, dtype=np.float64) / (s * (s - 1.0) / 2.0)
    Wc = (H.T @ sp.diags(pair) @ H).tocsr()
    Wc.setdiag(0.0)
    Wc.eliminate_zeros()
    return Wc


def dense_star_weights(n, m, eptr, pins, w) -> np.ndarray:
    """G_b's adjacency built entry by entry from the definition (small inputs)."""
    W = np.zeros((n + m, n + m))
    for e in range(m):
        mem = pins[eptr[e]:eptr[e + 1]]
        for p in mem:
            W[p, n + e] = W[n + e, p] = float(w[e]) / len(mem)
    return W


def dense_clique_weights(n, m, eptr, pins, w) -> np.ndarray:
    """G_c's adjacency built pair by pair from the definition (small inputs)."""
    W = np.zeros((n, n))
    for e in range(m):
        mem = [int(x) for x in pins[eptr[e]:eptr[e + 1]]]
        k = len(mem)
        share = float(w[e]) / (k * (k - 1) / 2)
        for a in range(k):
            for c in range(a + 1, k):
                W[mem[a], mem[c]] += share
                W[mem[c], mem[a]] += share
    return W


def normalized_adjacency(W):
    """D^-1/2 W D^-1/2 with D the weighted degrees; zero degree -> zero scale."""
    deg = np.asarray(W.sum(axis=1)).ravel()
    inv = np.zeros_like(deg)
    pos = deg > 0
    inv[pos] = 1.0 / np.sqrt(deg[pos])
    if sp.issparse(W):
        D = sp.diags(inv)
        return (D @ W @ D).tocsr()
    return inv[:, None] * W * inv[None, :]


def star_operator(n, m, eptr, pins, w):
    return normalized_adjacency(star_weights(n, m, eptr, pins, w))


def clique_operator(n, m, eptr, pins, w):
    return normalized_adjacency(clique_weights(n, m, eptr, pins, w))


# --------------------------------------------------------------------------
# Gram-Schmidt with column dropping (Alg. 1)
# --------------------------------------------------------------------------

def orthonormalize(V: np.ndarray, ref: np.ndarray, tau: float):
    """Gram-Schmidt of V's columns in order; a column whose residual is below
    tau * ref is dropped and the remaining columns are orthonormalised without
    it.  Returns (Q, kept column indices, |R_jj| of kept columns).
    Householder QR with the signs fixed so that diag(R) > 0 is the same
    factorisation as Gram-Schmidt."""
    cols = list(range(V.shape[1]))
    while cols:
        Q, R = np.linalg.qr(V[:, cols])
        d = np.zeros(len(cols))
        d[:min(R.shape)] = np.diag(R)       # columns past the row count have no residual
        ad = np.abs(d)
        bad = [j for j, c in enumerate(cols) if ref[c] == 0 or ad[j] < tau * ref[c]]
        if not bad:
            sgn = np.where(d < 0, -1.0, 1.0)
            return Q[:, :len(cols)] * sgn[None, :], np.asarray(cols), ad
        del cols[bad[0]]
    return np.zeros((V.shape[0], 0)), np.zeros(0, dtype=np.int64), np.zeros(0)


def krylov_blocks(A, X: np.ndarray, k: int, tau: float = 1e-3):
    """Orthonormal bases Q_0..Q_k of the block Krylov sequence X, AX, ..., A^k X
    (Eq. (12)); Q_j spans the part of A^j X orthogonal to the earlier blocks.
    Each new block is orthogonalised against all earlier ones twice
    (classical Gram-Schmidt, repeated)."""
    X = np.asarray(X, dtype=np.float64)
    Q0, _, _ = orthonormalize(X, np.linalg.norm(X, axis=0), tau)
    blocks = [Q0]
    total = Q0.shape[1]
    N = X.shape[0]
    basis = np.empty((N, X.shape[1] * (k + 1)))
    basis[:, :total] = Q0
    for _ in range(k):
        W = A @ blocks[-1]
        ref = np.linalg.norm(W, axis=0)
        B = basis[:, :total]
        for _rep in range(2):
            W = W - B @ (B.T @ W)
        Qj, _, _ = orthonormalize(W, ref, tau)
        blocks.append(Qj)
        basis[:, total:total + Qj.shape[1]] = Qj
        total += Qj.shape[1]
    return blocks


@dataclass
class Pool:
    chi: np.ndarray              # n x K_kept, orthonormal columns chi^(i)
    kept: np.ndarray             # indices of kept columns in the joint list
    rho: np.ndarray              # relative residuals |R_jj| / ||V_j|| of kept columns
    n_star: int                  # columns contributed by the star expansion
    n_clique: int
    star_blocks: list = field(default_factory=list)
    clique_blocks: list = field(default_factory=list)


def unified_pool(n, m, eptr, pins, w, X_star, X_clique, k, tau=1e-3,
                 use_star=True, use_clique=True, keep_blocks=True) -> Pool:
    """The pool chi^(1..2 rho) of Alg. 1: per-expansion Krylov bases
    without the start block, star vectors restricted to the hypergraph nodes,
    star columns first, then one joint Gram-Schmidt in R^n.  With
    keep_blocks=False the per-expansion blocks are released as soon as their
    pool columns are taken (same arithmetic, less host memory)."""
    cols = []
    sb, cb = [], []
    if use_star:
        Ab = star_operator(n, m, eptr, pins, w)
        sb = krylov_blocks(Ab, X_star, k, tau)
        cols += [np.ascontiguousarray(B[:n, :]) for B in sb[1:]]
        del Ab
        if not keep_blocks:
            sb = []
    ns = sum(c.shape[1] for c in cols)
    if use_clique:
        Ac = clique_operator(n, m, eptr, pins, w)
        cb = krylov_blocks(Ac, X_clique, k, tau)
        cols += [B for B in cb[1:]]
        del Ac
        if not keep_blocks:
            cb = []
    V = np.hstack(cols) if cols else np.zeros((n, 0))
    del cols
    Q, kept, rdiag = orthonormalize(V, np.linalg.norm(V, axis=0), tau)
    norms = np.linalg.norm(V, axis=0)
    rho = rdiag / norms[kept] if kept.size else rdiag
    return Pool(chi=Q, kept=kept, rho=rho, n_star=ns, n_clique=V.shape[1] - ns,
                star_blocks=sb, clique_blocks=cb)


# --------------------------------------------------------------------------
# Resistance ratios (Eqs. (9), (13), (14); Alg. 1)
# --------------------------------------------------------------------------

def edge_spread(eptr, pins, chi: np.ndarray) -> np.ndarray:
    """(max_{p in e} chi_p - min_{p in e} chi_p)^2 per hyperedge and column:
    the squared difference of the two most distant pins along chi."""
    eptr = np.asarray(eptr, dtype=np.int64)
    G = chi[np.asarray(pins, dtype=np.int64)]
    starts = eptr[:-1]
    d = np.maximum.reduceat(G, starts, axis=0) - np.minimum.reduceat(G, starts, axis=0)
    return d * d


def quadratic_forms(eptr, pins, w, chi: np.ndarray, chunk: int = 64) -> np.ndarray:
    """Q_H(chi^(i)) of Eq. (9) for every column i."""
    w = np.asarray(w, dtype=np.float64)
    K = chi.shape[1]
    out = np.zeros(K)
    for c0 in range(0, K, chunk):
        c1 = min(K, c0 + chunk)
        out[c0:c1] = w @ edge_spread(eptr, pins, chi[:, c0:c1])
    return out


def resistance_from_pool(eptr, pins, w, chi: np.ndarray, chunk: int = 64):
    """R_e = max_i (max-min)^2 / Q_H(chi^(i)) (Eqs. (13)-(14)) and Q_H per column."""
    qh = quadratic_forms(eptr, pins, w, chi, chunk)
    m = len(eptr) - 1
    R = np.zeros(m)
    usable = np.nonzero(qh > 0)[0]
    for c0 in range(0, usable.size, chunk):
        sel = usable[c0:c0 + chunk]
        r = edge_spread(eptr, pins, chi[:, sel]) / qh[sel][None, :]
        R = np.maximum(R, r.max(axis=1))
    return R, qh


@dataclass
class Estimate:
    R: np.ndarray
    qh: np.ndarray
    pool: Pool


def resistance(n, m, eptr, pins, w, X_star, X_clique, k, tau=1e-3, **kw) -> Estimate:
    """Alg. 1: hypergraph in, per-hyperedge effective-resistance estimates out."""
    pool = unified_pool(n, m, eptr, pins, w, X_star, X_clique, k, tau, **kw)
    R, qh = resistance_from_pool(eptr, pins, w, pool.chi)
    return Estimate(R=R, qh=qh, pool=pool)
