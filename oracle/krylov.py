"""Plain batched Krylov solvers for the projected shifted equations
(test infrastructure: part of the oracle).

Every column j solves A_j z = b_j with A_j = Q(H - s_j)Q, b_j in range(Q), from
z = 0.  For s_j <= eps_Ne < eps_{Ne+1} each A_j is positive definite on
range(Q), so conjugate gradients apply; MINRES is the solver the paper names
for these equations (Sec. 2.2, after Eq. (2.18); Paige and Saunders 1975).

Nothing is fused or reordered: each iteration applies the operator as written
(projector, Hamiltonian, shift, projector) and then the textbook recurrences.
"""
from __future__ import annotations

import numpy as np


def make_operator(model, veff, phi, shifts, H=None):
    """Column-wise A_j x = Q (H - s_j) Q x.  H: optionally the same Hamiltonian
    as a sparse matrix (model.hamiltonian_sparse(veff)), faster on large grids."""
    shifts = np.asarray(shifts, dtype=np.float64)

    def q(x):
        return x - phi @ (phi.T @ x)

    def apply(x):
        y = q(x)
        hy = model.hamiltonian_apply(veff, y) if H is None else H @ y
        y = hy - y * shifts[None, :]
        return q(y)

    return apply


def cg(apply_a, b, tol=1e-8, max_iter=5000):
    """Batched conjugate gradients; stops column j when ||r_j|| <= tol ||b_j||.
    Returns (x, iterations per column, recurrence residual norms)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.sum(r * r, axis=0)
    bnorm = np.sqrt(np.sum(b * b, axis=0))
    thresh = tol * bnorm
    active = np.sqrt(rr) > thresh
    iters = np.zeros(b.shape[1], dtype=np.int64)
    for _ in range(max_iter):
        if not active.any():
            break
        ap = apply_a(p)
        pap = np.sum(p * ap, axis=0)
        alpha = np.where(active, rr / np.where(active, pap, 1.0), 0.0)
        x += alpha * p
        r -= alpha * ap
        rr_new = np.sum(r * r, axis=0)
        beta = np.where(active, rr_new / np.where(active, rr, 1.0), 0.0)
        p = np.where(active, r + beta * p, p)
        rr = np.where(active, rr_new, rr)
        iters += active
        active = active & (np.sqrt(rr) > thresh)
    return x, iters, np.sqrt(rr)


def minres(apply_a, b, tol=1e-8, max_iter=5000):
    """Batched MINRES: Lanczos tridiagonalisation with the tridiagonal least-squares
    problem min || beta_1 e_1 - T_k y || reduced by Givens rotations; the
    solution is updated through the direction vectors W = V R^{-1}.
    Stops column j when the residual estimate |phibar| <= tol ||b_j||."""
    n, m = b.shape
    x = np.zeros_like(b)
    beta1 = np.sqrt(np.sum(b * b, axis=0))
    safe = np.where(beta1 > 0, beta1, 1.0)
    v = b / safe
    v_old = np.zeros_like(b)
    w = np.zeros_like(b)
    w_old = np.zeros_like(b)
    beta = beta1.copy()
    cs = -np.ones(m)
    sn = np.zeros(m)
    dbar = np.zeros(m)
    eps_next = np.zeros(m)
    phibar = beta1.copy()
    thresh = tol * beta1
    active = phibar > thresh
    iters = np.zeros(m, dtype=np.int64)
    for _ in range(max_iter):
        if not active.any():
            break
        av = apply_a(v)
        alpha = np.sum(v * av, axis=0)
        v_new = av - alpha * v - beta * v_old
        beta_new = np.sqrt(np.sum(v_new * v_new, axis=0))
        # previous rotations applied to the new column of T
        eps_k = eps_next
        delta = cs * dbar + sn * alpha
        gbar = sn * dbar - cs * alpha
        eps_next = sn * beta_new
        dbar = -cs * beta_new
        # new rotation annihilating beta_{k+1}
        gamma = np.sqrt(gbar * gbar + beta_new * beta_new)
        gamma = np.where(gamma > 0, gamma, 1e-300)
        cs_new = gbar / gamma
        sn_new = beta_new / gamma
        phi = cs_new * phibar
        w_new = (v - eps_k * w_old - delta * w) / gamma
        upd = active[None, :]
        x = np.where(upd, x + phi * w_new, x)
        phibar = np.where(active, sn_new * phibar, phibar)
        cs = np.where(active, cs_new, cs)
        sn = np.where(active, sn_new, sn)
        w_old = np.where(upd, w, w_old)
        w = np.where(upd, w_new, w)
        bsafe = np.where(beta_new > 0, beta_new, 1.0)
        v_old = np.where(upd, v, v_old)
        v = np.where(upd, v_new / bsafe, v)
        beta = np.where(active, beta_new, beta)
        iters += active
        active = active & (np.abs(phibar) > thresh)
    return x, iters, np.abs(phibar)


def true_residual(apply_a, x, b):
    """||b - A x|| / ||b|| per column; a zero column of b (whose solution is 0)
    reports the absolute residual ||A x||."""
    r = b - apply_a(x)
    rn = np.sqrt(np.sum(r * r, axis=0))
    bn = np.sqrt(np.sum(b * b, axis=0))
    return np.where(bn > 0, rn / np.where(bn > 0, bn, 1.0), rn)
