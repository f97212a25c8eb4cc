"""Derivative of L(w) = sum_e c_e R_e(w) with respect to the hyperedge weights.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The forward is Alg. 1 exactly as in ``oracle.resistance`` (same expansions,
same block Krylov sequences with repeated classical Gram-Schmidt against every
earlier block, same joint Gram-Schmidt, same ratios of Eqs. (9), (13), (14)),
re-expressed in float64 torch operations on the CPU so that autograd gives the
gradient.  The maxima are taken at explicit positions: the largest ratio at
the lowest column index, the largest / smallest pin at the lowest CSR
position; the derivative is the one of the branch those positions select.
Column dropping is not differentiated (the caller checks that nothing drops).
"""
from __future__ import annotations

import numpy as np
import torch


def _apply_star(n, m, eptr_t, pins_t, eid_t, w, X):
    """y = D^-1/2 W_b D^-1/2 x for the star expansion, W_b[e,p] = w_e/|e|."""
    size = (eptr_t[1:] - eptr_t[:-1]).to(torch.float64)
    z = w / size                                         # per hyperedge
    zp = z[eid_t]                                        # per pin
    deg_v = torch.zeros(n, dtype=torch.float64).index_add_(0, pins_t, zp)
    deg_e = torch.zeros(m, dtype=torch.float64).index_add_(0, eid_t, zp)
    sv = torch.where(deg_v > 0, deg_v.clamp_min(1e-300).rsqrt(), torch.zeros_like(deg_v))
    se = deg_e.rsqrt()
    xv, xe = X[:n], X[n:]
    ye = torch.zeros((m, X.shape[1]), dtype=torch.float64).index_add_(
        0, eid_t, (zp * sv[pins_t] * se[eid_t])[:, None] * xv[pins_t])
    yv = torch.zeros((n, X.shape[1]), dtype=torch.float64).index_add_(
        0, pins_t, (zp * sv[pins_t] * se[eid_t])[:, None] * xe[eid_t])
    return torch.cat([yv, ye], 0)


def _apply_clique(n, m, eptr_t, pins_t, eid_t, w, X):
    """y = D^-1/2 W_c D^-1/2 x for the clique expansion (no self loops)."""
    size = (eptr_t[1:] - eptr_t[:-1]).to(torch.float64)
    pair = w / (size * (size - 1) / 2)
    pp = pair[eid_t]
    deg = torch.zeros(n, dtype=torch.float64).index_add_(0, pins_t, pp * (size[eid_t] - 1))
    s = torch.where(deg > 0, deg.clamp_min(1e-300).rsqrt(), torch.zeros_like(deg))
    u = s[:, None] * X
    S = torch.zeros((m, X.shape[1]), dtype=torch.float64).index_add_(0, eid_t, u[pins_t])
    acc = torch.zeros((n, X.shape[1]), dtype=torch.float64).index_add_(
        0, pins_t, pp[:, None] * (S[eid_t] - u[pins_t]))
    return s[:, None] * acc


def _qr_pos(V):
    Q, R = torch.linalg.qr(V)
    sgn = torch.where(torch.diagonal(R) < 0, -1.0, 1.0).to(V.dtype)
    return Q * sgn[None, :]


def _krylov(apply, X, k):
    blocks = [_qr_pos(X)]
    for _ in range(k):
        W = apply(blocks[-1])
        B = torch.cat(blocks, 1)
        for _rep in range(2):
            W = W - B @ (B.T @ W)
        blocks.append(_qr_pos(W))
    return blocks


def resistance_torch(n, m, eptr, pins, w, X_star, X_clique, k):
    """Alg. 1 as a differentiable function of w (float64 tensor [m])."""
    eptr_t = torch.as_tensor(np.asarray(eptr, dtype=np.int64))
    pins_t = torch.as_tensor(np.asarray(pins, dtype=np.int64))
    eid_t = torch.repeat_interleave(torch.arange(m), eptr_t[1:] - eptr_t[:-1])
    sb = _krylov(lambda X: _apply_star(n, m, eptr_t, pins_t, eid_t, w, X),
                 torch.as_tensor(np.asarray(X_star, dtype=np.float64)), k)
    cb = _krylov(lambda X: _apply_clique(n, m, eptr_t, pins_t, eid_t, w, X),
                 torch.as_tensor(np.asarray(X_clique, dtype=np.float64)), k)
    V = torch.cat([B[:n] for B in sb[1:]] + cb[1:], 1)
    chi = _qr_pos(V)
    # per (e, i): positions of the largest and smallest pin
    G = chi[pins_t]                                     # nnz x K
    with torch.no_grad():
        starts = eptr_t[:-1]
        npins = pins_t.shape[0]
        pos = torch.arange(npins)
        big = torch.full((m, chi.shape[1]), -1, dtype=torch.int64)
        small = torch.full((m, chi.shape[1]), -1, dtype=torch.int64)
        Gd = G.detach().numpy()
        ep = np.asarray(eptr, dtype=np.int64)
        amax = np.stack([Gd[ep[e]:ep[e + 1]].argmax(0) for e in range(m)]) + ep[:-1, None]
        amin = np.stack([Gd[ep[e]:ep[e + 1]].argmin(0) for e in range(m)]) + ep[:-1, None]
        big = torch.as_tensor(amax)
        small = torch.as_tensor(amin)
        del starts, pos
    cols = torch.arange(chi.shape[1])[None, :].expand(m, -1)
    spread = (G[big, cols] - G[small, cols]) ** 2          # m x K
    qh = (w[:, None] * spread).sum(0)
    ratio = spread / qh[None, :]
    with torch.no_grad():
        arg = ratio.argmax(1)                              # first maximum
    R = ratio[torch.arange(m), arg]
    return R, qh, chi


def loss_and_grad(n, m, eptr, pins, w, X_star, X_clique, k, coef):
    """L = sum_e coef_e R_e and dL/dw (float64 numpy)."""
    wt = torch.tensor(np.asarray(w, dtype=np.float64), requires_grad=True)
    R, _, _ = resistance_torch(n, m, eptr, pins, wt, X_star, X_clique, k)
    L = (torch.as_tensor(np.asarray(coef, dtype=np.float64)) * R).sum()
    L.backward()
    return float(L.detach()), wt.grad.numpy().copy(), R.detach().numpy()
