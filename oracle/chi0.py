"""Exact linear response (test infrastructure: part of the oracle).

* chi0 by the Adler-Wiser sum over states (Sec. 2.2, Eq. (2.17)), in the
  discrete normalisation: as a matrix acting on grid potentials
      X0 = (2 f / h^d) sum_{i<=N_e} sum_{a>N_e} (phi_i o phi_a)(phi_i o phi_a)^T / (eps_i - eps_a)
  with l2-orthonormal grid eigenvectors phi and f electrons per orbital.
* chi0 g by the Sternheimer form (Eq. (2.18), Alg. 1) with the projected
  shifted equations solved by dense factorisation -- a second, independent
  formula for the same quantity.
* chi = (I - chi0 v_hxc)^{-1} chi0 (Eq. (2.14)) with v_hxc = v_c (no xc kernel)
  by a dense solve; the Neumann fixed point of Eq. (2.16) for comparison.
* The Hessian of Eq. (2.11): h^d g_I^T (chi g_J) + local terms.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .model import Model, GroundState


def full_spectrum(model: Model, gs: GroundState):
    """All eigenpairs of H[V_eff] (dense eigh; small grids only)."""
    H = model.hamiltonian_dense(gs.veff)
    w, v = np.linalg.eigh(H)
    return w, v


def chi0_sos_matrix(model: Model, w: np.ndarray, v: np.ndarray, n_e: int) -> np.ndarray:
    """Dense X0 by the sum over states, Eq. (2.17)."""
    pref = 2.0 * model.f / model.grid.dv
    occ, unocc = v[:, :n_e], v[:, n_e:]
    n_g = v.shape[0]
    X0 = np.zeros((n_g, n_g))
    for i in range(n_e):
        P = occ[:, i:i + 1] * unocc                    # columns phi_i o phi_a
        den = 1.0 / (w[i] - w[n_e:])
        X0 += pref * (P * den[None, :]) @ P.T
    return X0


def chi0_apply_sos(model: Model, w, v, n_e: int, g: np.ndarray) -> np.ndarray:
    """X0 g by the sum over states without forming X0 (any number of columns)."""
    pref = 2.0 * model.f / model.grid.dv
    occ, unocc = v[:, :n_e], v[:, n_e:]
    g2 = g.reshape(g.shape[0], -1)
    out = np.zeros_like(g2)
    for i in range(n_e):
        c = unocc.T @ (occ[:, i:i + 1] * g2)
        c /= (w[i] - w[n_e:])[:, None]
        out += pref * occ[:, i:i + 1] * (unocc @ c)
    return out.reshape(g.shape)


def chi0_apply_sternheimer(model: Model, gs: GroundState, g: np.ndarray) -> np.ndarray:
    """Alg. 1: chi0 g = 2f/h^d sum_i phi_i o zeta_i,  Q(eps_i - H)Q zeta_i = Q(phi_i o g).

    Each projected equation is solved densely on range(Q) through the
    nonsingular matrix Q(eps_i - H)Q + Phi Phi^T, whose solution for a
    right-hand side in range(Q) lies in range(Q).
    """
    pref = 2.0 * model.f / model.grid.dv
    phi = gs.phi
    n_e = gs.n_e
    H = model.hamiltonian_dense(gs.veff)
    n_g = H.shape[0]
    Q = np.eye(n_g) - phi @ phi.T
    P = phi @ phi.T
    g2 = g.reshape(n_g, -1)
    out = np.zeros_like(g2)
    for i in range(n_e):
        A = Q @ (gs.eps[i] * np.eye(n_g) - H) @ Q + P
        rhs = Q @ (phi[:, i:i + 1] * g2)
        zeta = np.linalg.solve(A, rhs)
        out += pref * phi[:, i:i + 1] * zeta
    return out.reshape(g.shape)


def dyson_dense(X0: np.ndarray, Vc: np.ndarray, G: np.ndarray) -> np.ndarray:
    """U = chi G with chi = (I - X0 v_c)^{-1} X0  (Eq. (2.14))."""
    n = X0.shape[0]
    return np.linalg.solve(np.eye(n) - X0 @ Vc, X0 @ G)


def dyson_neumann(X0: np.ndarray, Vc: np.ndarray, G: np.ndarray, n_iter: int) -> np.ndarray:
    """Fixed point u^{k+1} = chi0 g + chi0 v u^k of Eq. (2.16), from u^0 = 0."""
    X0G = X0 @ G
    K = X0 @ Vc
    u = np.zeros_like(G)
    for _ in range(n_iter):
        u = X0G + K @ u
    return u


def hessian_exact(model: Model, gs: GroundState, U: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Eq. (2.11): h^d G^T U + local terms (pseudocharge form)."""
    return model.grid.dv * (G.T @ U) + model.local_hessian(gs)


def dynamical_matrix(hess: np.ndarray, masses: np.ndarray, dim: int):
    """D = M^{-1/2} Hess M^{-1/2} (Sec. 2.2) and its eigenvalues omega_k^2 (ascending).

    The Hessian is symmetrised first.  masses has one entry per atom.
    """
    hs = 0.5 * (hess + hess.T)
    minv = np.repeat(1.0 / np.sqrt(np.asarray(masses, dtype=np.float64)), dim)
    D = minv[:, None] * hs * minv[None, :]
    lam = np.linalg.eigvalsh(D)
    return D, lam


def phonon_dos(omega2: np.ndarray, n_modes: int, sigma: float, w: np.ndarray) -> np.ndarray:
    """Phonon spectrum rho_D(w) = (1 / (d N_A)) sum_k delta_sigma(w - w_k) (Sec. 2.2),
    the delta replaced by the normalised Gaussian of width sigma as in Sec. 4;
    w_k = sign(omega_k^2) sqrt(|omega_k^2|) (a slightly negative omega^2 from
    rounding becomes a small negative frequency).  n_modes = d N_A."""
    wk = np.sign(omega2) * np.sqrt(np.abs(omega2))
    x = np.asarray(w, dtype=np.float64)[:, None] - wk[None, :]
    g = np.exp(-x ** 2 / (2.0 * sigma ** 2)) / np.sqrt(2.0 * np.pi * sigma ** 2)
    return g.sum(axis=1) / n_modes

