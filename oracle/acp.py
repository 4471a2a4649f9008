"""The ACP method step by step (test infrastructure: part of the oracle).

Follows Sec. 3 of the paper in its own order and notation:

  Chebyshev nodes on [eps_1, eps_Ne] and Lagrange weights      Sec. 3.1, Eq. (3.4)
  interpolative decomposition of M (Alg. 2, sketched as in the Remark after it)
  right-hand sides Q xi_mu and the compressed shifted equations  Eq. (3.6)
  W by Chebyshev interpolation in the shift                      Eq. (3.7)
  chi0~ = W Pi^T                                                 Eq. (3.9)
  adaptive compression of the Dyson equation with the
  Sherman-Morrison-Woodbury update                              Alg. 4, Eq. (3.13)
  dynamical matrix and phonon frequencies                        Sec. 2.2

Readings where the paper is silent or garbled (also listed in the design notes):
  * the sketch is the Remark's variant: G~ = G Omega with a real Gaussian Omega
    (n_p x r) supplied by the caller; rows of M~ are the Kronecker products
    G~(alpha, :) x phi(alpha, :);
  * pivoted QR is LAPACK's column-pivoted QR (a library primitive); the rank is
    the fixed N_mu unless a threshold is given (Alg. 2, step 3);
  * Eq. (3.7) lacks the mu index on zeta~ and is read as
      W_mu = (2 f / h^d) sum_c zeta~_{c mu} o [Phi diag(L_c(eps)) Phi(Pi,:)^T]_{:, mu};
  * the shifted equations are written in their positive-definite form
      Q(H - eps~_c)Q zeta = -Q xi,  equivalent to Q(eps~_c - H)Q zeta = Q xi;
  * Dyson stopping: relative Frobenius change of U = U~ - B;
    iteration 0 compresses v_hxc U~^0 = v_c B = G exactly.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------------
# Sec. 3.1: shifts and interpolation weights
# ----------------------------------------------------------------------------
def chebyshev_nodes(eps_lo: float, eps_hi: float, n_c: int) -> np.ndarray:
    """eps~_c = (eps_1 + eps_Ne)/2 + (eps_1 - eps_Ne)/2 cos(pi (c - 1/2) / N_c), c = 1..N_c."""
    c = np.arange(1, n_c + 1)
    theta = np.pi * (c - 0.5) / n_c
    return 0.5 * (eps_lo + eps_hi) + 0.5 * (eps_lo - eps_hi) * np.cos(theta)


def lagrange_weights(nodes: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """L[c, i] = prod_{c' != c} (eps_i - eps~_c') / (eps~_c - eps~_c')  (Eq. (3.4))."""
    n_c = len(nodes)
    L = np.ones((n_c, len(eps)))
    for c in range(n_c):
        for cp in range(n_c):
            if cp != c:
                L[c] *= (eps - nodes[cp]) / (nodes[c] - nodes[cp])
    return L


# ----------------------------------------------------------------------------
# Alg. 2: interpolative decomposition of M (sketched)
# ----------------------------------------------------------------------------
def sketched_rows(phi: np.ndarray, G: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """M~ (N_g x r N_e): row alpha is G~(alpha, :) (x) phi(alpha, :), G~ = G Omega."""
    Gt = G @ omega
    n_g = phi.shape[0]
    return (Gt[:, :, None] * phi[:, None, :]).reshape(n_g, -1)


@dataclasses.dataclass
class ISDF:
    sel: np.ndarray        # selected grid indices r_mu (in pivot order)
    xi: np.ndarray         # N_g x N_mu interpolation vectors
    rdiag: np.ndarray      # |R~_kk| of the pivoted QR (empty when the selection is forced)


def isdf_qrcp(phi: np.ndarray, G: np.ndarray, omega: np.ndarray, n_mu: int,
              tol: float = 0.0) -> ISDF:
    """Alg. 2 steps 2-4: pivoted QR of M~^T, rank rule, Xi^T = R11^{-1} R_{1:N_mu,:} Pi~^{-1}."""
    Mt = sketched_rows(phi, G, omega)
    _, R, piv = sla.qr(Mt.T, mode="economic", pivoting=True)
    rd = np.abs(np.diag(R))
    if tol > 0:
        small = np.nonzero(rd < tol * rd[0])[0]
        if small.size:
            n_mu = min(n_mu, int(small[0]))
    if n_mu > R.shape[0]:
        raise ValueError("N_mu exceeds the rank bound r N_e of the sketch")
    coef = sla.solve_triangular(R[:n_mu, :n_mu], R[:n_mu, :])   # N_mu x N_g, pivoted order
    xiT = np.empty_like(coef)
    xiT[:, piv] = coef
    xi = np.ascontiguousarray(xiT.T)
    sel = piv[:n_mu].copy()
    xi[sel, :] = np.eye(n_mu)
    return ISDF(sel=sel, xi=xi, rdiag=rd)


def isdf_forced(phi: np.ndarray, G: np.ndarray, omega: np.ndarray, sel: np.ndarray) -> ISDF:
    """Interpolation vectors for a given selection: the least-squares coefficients
    that reproduce every row of M~ from the selected rows,
      Xi^T = argmin_X || M~(sel, :)^T X - M~^T ||,
    which equals R11^{-1} R12 of a pivoted QR whose leading pivots are sel."""
    Mt = sketched_rows(phi, G, omega)
    A1 = Mt[sel, :].T
    X, *_ = np.linalg.lstsq(A1, Mt.T, rcond=None)
    xi = np.ascontiguousarray(X.T)
    xi[sel, :] = np.eye(len(sel))
    return ISDF(sel=np.asarray(sel).copy(), xi=xi, rdiag=np.empty(0))


def id_residual(phi, G, omega, isdf: ISDF) -> float:
    """|| M~ - Xi M~(sel, :) ||_F (the interpolation error of Eq. (3.5) on the sketch)."""
    Mt = sketched_rows(phi, G, omega)
    return float(np.linalg.norm(Mt - isdf.xi @ Mt[isdf.sel, :]))


# ----------------------------------------------------------------------------
# Eq. (3.6): right-hand sides and exact solutions of the compressed equations
# ----------------------------------------------------------------------------
def project_q(phi: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Q X = X - Phi (Phi^T X)."""
    return X - phi @ (phi.T @ X)


def rhs(phi: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Right-hand sides of the positive-definite form: -Q xi_mu (N_g x N_mu)."""
    return -project_q(phi, xi)


class ExactShiftedSolver:
    """Solves Q(H - s)Q z = b, b in range(Q), exactly from the full spectrum of H:
    z = sum_{a > N_e} phi_a (phi_a^T b) / (eps_a - s)."""

    def __init__(self, w: np.ndarray, v: np.ndarray, n_e: int):
        self.wu = w[n_e:]
        self.vu = v[:, n_e:]

    def __call__(self, shift: float, b: np.ndarray) -> np.ndarray:
        c = self.vu.T @ b
        c /= (self.wu - shift)[:, None]
        return self.vu @ c


class DenseShiftedSolver:
    """Same solution by a dense factorisation of Q(H - s)Q + Phi Phi^T (no spectrum)."""

    def __init__(self, H: np.ndarray, phi: np.ndarray):
        self.H = H
        self.phi = phi

    def __call__(self, shift: float, b: np.ndarray) -> np.ndarray:
        n = self.H.shape[0]
        P = self.phi @ self.phi.T
        Q = np.eye(n) - P
        A = Q @ (self.H - shift * np.eye(n)) @ Q + P
        return np.linalg.solve(A, b)


class ProjectedSpectralSolver:
    """Same solution for any l2-orthonormal Phi (not necessarily eigenvectors of
    H) from the eigenpairs of Q H Q + c Phi Phi^T, c above the spectrum of H:
    its eigenvectors with eigenvalues below c span range(Q), so
    z = sum_{mu_a < c} u_a (u_a^T b) / (mu_a - s)."""

    def __init__(self, H: np.ndarray, phi: np.ndarray):
        n = H.shape[0]
        P = phi @ phi.T
        Q = np.eye(n) - P
        c = 2.0 * np.abs(H).sum(axis=1).max() + 1.0   # Gershgorin bound, doubled
        mu, U = np.linalg.eigh(Q @ H @ Q + c * P)
        keep = mu < 0.5 * c
        self.mu, self.U = mu[keep], U[:, keep]

    def __call__(self, shift: float, b: np.ndarray) -> np.ndarray:
        y = self.U.T @ b
        y /= (self.mu - shift)[:, None]
        return self.U @ y


def solve_compressed(solver: Callable, nodes: np.ndarray, R: np.ndarray) -> List[np.ndarray]:
    """Z_c (N_g x N_mu) for every shift eps~_c: Q(H - eps~_c)Q Z_c = R."""
    return [solver(float(s), R) for s in nodes]


def assemble_w(phi: np.ndarray, L: np.ndarray, sel: np.ndarray, Z: List[np.ndarray],
               f: float, dv: float) -> np.ndarray:
    """Eq. (3.7): W = (2f/h^d) sum_c Z_c o (Phi diag(L_c) Phi(sel,:)^T)."""
    W = np.zeros_like(Z[0])
    for c, Zc in enumerate(Z):
        W += Zc * (phi @ (L[c][:, None] * phi[sel, :].T))
    return (2.0 * f / dv) * W


def chi0_tilde_apply(W: np.ndarray, sel: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Eq. (3.9): chi0~ X = W Pi^T X = W X(sel, :)."""
    return W @ X[sel, :]


# ----------------------------------------------------------------------------
# Alg. 3 and Alg. 4
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Compressed:
    sel: np.ndarray
    xi: np.ndarray
    R: np.ndarray
    Z: List[np.ndarray]
    W: np.ndarray


def compress(phi, eps_occ, G, omega, n_c, n_mu, solver, f, dv, *, sel=None,
             node_mode: str = "chebyshev", isdf_tol: float = 0.0) -> Compressed:
    """Alg. 3: chi0~ = W Pi^T for the columns of G."""
    if sel is None:
        dec = isdf_qrcp(phi, G, omega, n_mu, tol=isdf_tol)
    else:
        dec = isdf_forced(phi, G, omega, np.asarray(sel))
    nodes, L = shifts_and_weights(eps_occ, n_c, node_mode)
    R = rhs(phi, dec.xi)
    Z = solve_compressed(solver, nodes, R)
    W = assemble_w(phi, L, dec.sel, Z, f, dv)
    return Compressed(sel=dec.sel, xi=dec.xi, R=R, Z=Z, W=W)


def shifts_and_weights(eps_occ: np.ndarray, n_c: int, node_mode: str = "chebyshev"):
    """Nodes and weights; a degenerate interval collapses to one node with L = 1.
    node_mode 'occupied' uses the distinct occupied eigenvalues themselves as
    nodes, for which the interpolation is exact."""
    eps_occ = np.asarray(eps_occ, dtype=np.float64)
    lo, hi = float(eps_occ[0]), float(eps_occ[-1])
    if node_mode == "occupied":
        nodes = np.unique(eps_occ)
    elif hi - lo <= 1e-14 * max(1.0, abs(lo)) or n_c == 1:
        nodes = np.array([0.5 * (lo + hi)])
    else:
        nodes = chebyshev_nodes(lo, hi, n_c)
    if len(nodes) == 1:
        return nodes, np.ones((1, len(eps_occ)))
    return nodes, lagrange_weights(nodes, eps_occ)


@dataclasses.dataclass
class DysonResult:
    U: np.ndarray
    iters: int
    sel_hist: List[np.ndarray]
    W_hist: List[np.ndarray]
    changes: List[float]
    last: Optional[Compressed] = None   # the last compression (Z, W, selection)


def acp_dyson(phi, eps_occ, G, omega, n_c, n_mu, solver, *, vc: Callable, vc_inv: Callable,
              f: float, dv: float, k_max: int = 4, delta: float = 0.0,
              sel_hist: Optional[List[np.ndarray]] = None, node_mode: str = "chebyshev",
              isdf_tol: float = 0.0) -> DysonResult:
    """Alg. 4 with the update of Eq. (3.13):
        B = v_hxc^{-1} G,  U~^0 = B
        repeat: compress v_hxc U~^k -> W^k, Pi^k
                U~^{k+1} = B + W^k (I - Pi^T v W^k)^{-1} Pi^T v B
        U = U~ - B.
    With v_hxc = v_c:  Pi^T v B = G(Pi, :)  and  v_hxc U~^{k+1} = G + (v_c W^k) S^k,
    S^k = (I - (v_c W^k)(Pi^k, :))^{-1} G(Pi^k, :), so U^{k+1} = W^k S^k.
    Stops after k_max compressions or when ||U^{k+1} - U^k||_F <= delta ||U^{k+1}||_F.
    """
    _ = vc_inv  # B itself is not needed once U = W S is formed directly
    Gk = G.copy()
    U_prev = np.zeros_like(G)
    sels, Ws, changes = [], [], []
    it = 0
    last = None
    for it in range(1, k_max + 1):
        forced = None if sel_hist is None else sel_hist[it - 1]
        comp = compress(phi, eps_occ, Gk, omega, n_c, n_mu, solver, f, dv, sel=forced,
                        node_mode=node_mode, isdf_tol=isdf_tol)
        V = vc(comp.W)
        T = V[comp.sel, :]
        S = np.linalg.solve(np.eye(len(comp.sel)) - T, G[comp.sel, :])
        U = comp.W @ S
        Gk = G + V @ S
        ch = np.linalg.norm(U - U_prev) / max(np.linalg.norm(U), 1e-300)
        sels.append(comp.sel)
        Ws.append(comp.W)
        changes.append(float(ch))
        U_prev = U
        last = comp
        if delta > 0 and ch <= delta:
            break
    return DysonResult(U=U_prev, iters=it, sel_hist=sels, W_hist=Ws, changes=changes, last=last)


def smw_dense_reference(W, sel, Vc_dense, B) -> np.ndarray:
    """(I - W Pi^T v_c)^{-1} B by a dense solve: the left side of Eq. (3.13)."""
    n = W.shape[0]
    P = np.zeros((n, len(sel)))
    P[sel, np.arange(len(sel))] = 1.0
    return np.linalg.solve(np.eye(n) - W @ P.T @ Vc_dense, B)
