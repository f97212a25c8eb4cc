"""Exact quantities the estimate is bounded by (small inputs only).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

* Eq. (6): graph effective resistance R_eff(p, q) = b_pq^T L^+ b_pq from the
  Moore-Penrose pseudo-inverse of the Laplacian L = D - A of Eq. (1).
* Eq. (8): the exact hyperedge resistance diameter
  R*_e = max_{p,q in e} max_chi (chi_p - chi_q)^2 / Q_H(chi), i.e.
  max_{p,q in e} 1 / min { Q_H(chi) : chi_p - chi_q = 1 }, a convex program
  (Q_H of Eq. (9) is a weighted sum of maxima of convex quadratics).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def laplacian(W: np.ndarray) -> np.ndarray:
    return np.diag(W.sum(axis=1)) - W


def pinv_resistance(W: np.ndarray) -> np.ndarray:
    """All-pairs R_eff(p, q) = (e_p - e_q)^T L^+ (e_p - e_q) (Eq. (6))."""
    Lp = np.linalg.pinv(laplacian(W))
    d = np.diag(Lp)
    return d[:, None] + d[None, :] - 2 * Lp


def max_pair(Reff: np.ndarray, eptr, pins) -> np.ndarray:
    """max_{p,q in e} Reff[p, q] for every hyperedge."""
    out = np.zeros(len(eptr) - 1)
    for e in range(len(eptr) - 1):
        mem = np.asarray(pins[eptr[e]:eptr[e + 1]], dtype=np.int64)
        out[e] = Reff[np.ix_(mem, mem)].max()
    return out


def q_h(eptr, pins, w, chi: np.ndarray) -> float:
    """Eq. (9) by brute force over all pairs of every hyperedge."""
    tot = 0.0
    for e in range(len(eptr) - 1):
        mem = chi[np.asarray(pins[eptr[e]:eptr[e + 1]], dtype=np.int64)]
        tot += float(w[e]) * float(((mem[:, None] - mem[None, :]) ** 2).max())
    return tot


def min_q_h_unit_gap(n, eptr, pins, w, p, q, restarts: int = 3, seed: int = 0) -> float:
    """min Q_H(chi) subject to chi_p - chi_q = 1.

    Written as min sum_e w_e g_e^2 over (chi, g) with g_e >= chi_u - chi_v for
    every ordered pin pair of e -- a convex QP with linear constraints."""
    m = len(eptr) - 1
    cons_rows = []
    for e in range(m):
        mem = [int(x) for x in pins[eptr[e]:eptr[e + 1]]]
        for u in mem:
            for v in mem:
                if u != v:
                    cons_rows.append((e, u, v))
    A = np.zeros((len(cons_rows), n + m))
    for r, (e, u, v) in enumerate(cons_rows):
        A[r, n + e] = 1.0      # g_e - chi_u + chi_v >= 0
        A[r, u] -= 1.0
        A[r, v] += 1.0
    wv = np.asarray(w, dtype=np.float64)

    def f(x):
        g = x[n:]
        return float((wv * g * g).sum())

    def grad(x):
        out = np.zeros_like(x)
        out[n:] = 2 * wv * x[n:]
        return out

    cons = [{"type": "ineq", "fun": lambda x: A @ x, "jac": lambda x: A},
            {"type": "eq", "fun": lambda x: np.array([x[p] - x[q] - 1.0]),
             "jac": lambda x: np.eye(n + m)[[p]] - np.eye(n + m)[[q]]}]
    rng = np.random.default_rng(seed)
    best = np.inf
    for _ in range(restarts):
        chi0 = rng.standard_normal(n)
        chi0[p], chi0[q] = 0.5, -0.5
        g0 = np.zeros(m)
        for e in range(m):
            mem = chi0[np.asarray(pins[eptr[e]:eptr[e + 1]], dtype=np.int64)]
            g0[e] = mem.max() - mem.min()
        res = minimize(f, np.concatenate([chi0, g0]), jac=grad, constraints=cons,
                       method="SLSQP", options={"maxiter": 500, "ftol": 1e-12})
        if res.success:
            best = min(best, res.fun)
    return best


def exact_resistance_diameter(n, eptr, pins, w, e: int) -> float:
    """R*_e of Eq. (8)."""
    mem = [int(x) for x in pins[eptr[e]:eptr[e + 1]]]
    best = 0.0
    for a in range(len(mem)):
        for c in range(a + 1, len(mem)):
            best = max(best, 1.0 / min_q_h_unit_gap(n, eptr, pins, w, mem[a], mem[c]))
    return best
