"""Discrete model of the paper (test infrastructure: part of the oracle).

The continuous model is the Kohn-Sham / reduced Hartree-Fock functional of
Sec. 2.1 (Eq. (2.1)) with the exchange-correlation term dropped as in the 1D
model of Sec. 4.1 (Eq. (4.1)), ions represented by Gaussian pseudocharges
(Eq. (2.3), Eq. (4.2)) and the Coulomb kernel replaced by the Yukawa kernel
whose defining equation is Eq. (4.4):  (-Delta + kappa^2) K = (4 pi / eps0) delta.

Discretisation (readings where the paper is silent; it used planewaves):
  * periodic uniform grid, spacing h, N_g points, index alpha = ix + nx * iy;
  * Delta_h = 8th-order central finite-difference Laplacian (per axis
    h^-2 * sum_{s=-4..4} c_|s| u_{alpha + s e});
  * v_c = (4 pi / eps0) (-Delta_h + kappa^2)^{-1}, applied exactly by FFT with
    the symbol of Delta_h, so that v_c^{-1} is the stencil itself;
  * orbitals phi_i are l2-orthonormal grid vectors (phi = psi * h^{d/2});
    rho = (f / h^d) sum_i phi_i^2 with f electrons per orbital;
  * integrals become h^d * sums.

All arithmetic is FP64 numpy/scipy.  Nothing here is shared with the HIP path.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.linalg as sla

# Central 8th-order coefficients of the second derivative, c_0 .. c_4.
FD8 = np.array([-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0])


# ----------------------------------------------------------------------------
# Grid operators
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Grid:
    n: tuple          # points per axis (x first)
    h: float

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def n_grid(self) -> int:
        return int(np.prod(self.n))

    @property
    def dv(self) -> float:
        return self.h ** self.dim

    @property
    def box(self) -> tuple:
        return tuple(k * self.h for k in self.n)

    def shape_c(self):
        """C-order array shape with x fastest: (ny, nx) in 2D, (nx,) in 1D."""
        return tuple(reversed(self.n))

    def coords(self):
        """Coordinates (N_g x d) of the grid points, alpha = ix + nx * iy."""
        axes = [np.arange(k) * self.h for k in self.n]
        mesh = np.meshgrid(*axes, indexing="ij")
        return np.stack([m.ravel(order="F") for m in mesh], axis=1)


def laplacian_apply(grid: Grid, u: np.ndarray) -> np.ndarray:
    """Delta_h u for u of shape (N_g,) or (N_g, k): periodic 8th-order stencil."""
    extra = u.shape[1:]
    uu = u.reshape(grid.shape_c() + extra)
    out = np.zeros_like(uu)
    for axis in range(grid.dim):
        ax = grid.dim - 1 - axis  # x is the last C axis
        out += FD8[0] * uu
        for s in range(1, 5):
            out += FD8[s] * (np.roll(uu, s, axis=ax) + np.roll(uu, -s, axis=ax))
    return (out / grid.h ** 2).reshape(u.shape)


def laplacian_dense(grid: Grid) -> np.ndarray:
    """Dense N_g x N_g matrix of Delta_h (only for small grids)."""
    return laplacian_apply(grid, np.eye(grid.n_grid))


def fd_symbol_1d(n: int, h: float) -> np.ndarray:
    """Eigenvalues of -Delta_h (one axis) on the Fourier modes k = 0..n-1.

    For u_j = exp(i theta j), theta = 2 pi k / n, the stencil gives
    h^-2 (c_0 + 2 sum_s c_s cos(s theta)) u, so -Delta_h has the eigenvalue
    h^-2 (-c_0 - 2 sum_s c_s cos(s theta)) >= 0.
    """
    theta = 2.0 * np.pi * np.arange(n) / n
    lam = -FD8[0] - 2.0 * sum(FD8[s] * np.cos(s * theta) for s in range(1, 5))
    return lam / h ** 2


def neg_laplacian_symbol(grid: Grid) -> np.ndarray:
    """Symbol of -Delta_h on the FFT grid of shape grid.shape_c()."""
    lam = [fd_symbol_1d(k, grid.h) for k in grid.n]
    if grid.dim == 1:
        return lam[0]
    return lam[1][:, None] + lam[0][None, :]


def yukawa_apply(grid: Grid, kappa: float, eps0: float, x: np.ndarray) -> np.ndarray:
    """v_c x with v_c = (4 pi / eps0) (-Delta_h + kappa^2)^{-1}, exact by FFT."""
    extra = x.shape[1:]
    xx = x.reshape(grid.shape_c() + extra)
    axes = tuple(range(grid.dim))
    sym = (4.0 * np.pi / eps0) / (neg_laplacian_symbol(grid) + kappa ** 2)
    sym = sym.reshape(sym.shape + (1,) * len(extra))
    y = np.fft.ifftn(np.fft.fftn(xx, axes=axes) * sym, axes=axes).real
    return y.reshape(x.shape)


def yukawa_inverse_apply(grid: Grid, kappa: float, eps0: float, x: np.ndarray) -> np.ndarray:
    """v_c^{-1} x = (eps0 / 4 pi) (-Delta_h x + kappa^2 x): a stencil."""
    return (eps0 / (4.0 * np.pi)) * (-laplacian_apply(grid, x) + kappa ** 2 * x)


def yukawa_dense(grid: Grid, kappa: float, eps0: float) -> np.ndarray:
    return yukawa_apply(grid, kappa, eps0, np.eye(grid.n_grid))


# ----------------------------------------------------------------------------
# Pseudocharges (Eq. (2.3), Eq. (4.2))
# ----------------------------------------------------------------------------
def min_image(grid: Grid, R: np.ndarray) -> np.ndarray:
    """Displacements r_alpha - R_I (N_g x N_A x d), minimum image convention."""
    X = grid.coords()
    L = np.array(grid.box)
    D = X[:, None, :] - R[None, :, :]
    return D - L * np.round(D / L)


def pseudocharges(grid: Grid, R: np.ndarray, Z: np.ndarray, sigma: float):
    """Gaussian pseudocharges and their derivatives with respect to R.

    m_I(r) = -Z_I (2 pi sigma^2)^{-d/2} exp(-|r - R_I|^2 / (2 sigma^2)).
    Returns
      m_each  (N_g x N_A)        the individual m_I
      dm      (N_g x d N_A)      d m_I / d R_{I,a}, column j = a + d * I
      d2m     (N_g x N_A x d x d) d^2 m_I / d R_{I,a} d R_{I,b}
    """
    d = grid.dim
    D = min_image(grid, R)                       # N_g x N_A x d
    r2 = np.sum(D * D, axis=2)
    pref = -Z[None, :] * (2.0 * np.pi * sigma ** 2) ** (-d / 2.0)
    m_each = pref * np.exp(-r2 / (2.0 * sigma ** 2))
    dm = m_each[:, :, None] * D / sigma ** 2     # N_g x N_A x d
    eye = np.eye(d)
    d2m = m_each[:, :, None, None] * (D[:, :, :, None] * D[:, :, None, :] / sigma ** 4
                                      - eye[None, None] / sigma ** 2)
    n_g, n_a = m_each.shape
    dm_cols = dm.reshape(n_g, n_a * d)           # j = a + d * I
    return m_each, dm_cols, d2m


# ----------------------------------------------------------------------------
# Model container, SCF ground state
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class GroundState:
    phi: np.ndarray       # N_g x N_e, l2-orthonormal occupied orbitals
    eps: np.ndarray       # N_e + n_extra lowest eigenvalues (ascending)
    veff: np.ndarray      # N_g
    rho: np.ndarray       # N_g
    n_e: int
    scf_iters: int
    scf_residual: float

    @property
    def gap(self) -> float:
        return float(self.eps[self.n_e] - self.eps[self.n_e - 1])


class Model:
    """Discrete model for given sites R (N_A x d) and charges Z."""

    def __init__(self, grid: Grid, R: np.ndarray, Z: np.ndarray, n_e: int, *,
                 sigma: float, kappa: float, eps0: float, f: float):
        self.grid = grid
        self.R = np.asarray(R, dtype=np.float64).reshape(-1, grid.dim)
        self.Z = np.asarray(Z, dtype=np.float64)
        self.n_e = int(n_e)
        self.sigma, self.kappa, self.eps0, self.f = sigma, kappa, eps0, f
        self.m_each, self.dm, self.d2m = pseudocharges(grid, self.R, self.Z, sigma)
        self.m = self.m_each.sum(axis=1)

    # -- operators ---------------------------------------------------------
    @property
    def n_atoms(self) -> int:
        return self.R.shape[0]

    def vc(self, x):
        return yukawa_apply(self.grid, self.kappa, self.eps0, x)

    def vc_inv(self, x):
        return yukawa_inverse_apply(self.grid, self.kappa, self.eps0, x)

    def hamiltonian_dense(self, veff: np.ndarray) -> np.ndarray:
        H = -0.5 * laplacian_dense(self.grid)
        H[np.diag_indices_from(H)] += veff
        return H

    def hamiltonian_apply(self, veff: np.ndarray, x: np.ndarray) -> np.ndarray:
        vv = veff if x.ndim == 1 else veff[:, None]
        return -0.5 * laplacian_apply(self.grid, x) + vv * x

    def density(self, phi: np.ndarray) -> np.ndarray:
        return (self.f / self.grid.dv) * np.sum(phi * phi, axis=1)

    def veff_of(self, rho: np.ndarray) -> np.ndarray:
        """Eq. (2.7) without V_xc: V = v_c (rho + m)."""
        return self.vc(rho + self.m)

    def lowest_eigenpairs(self, veff: np.ndarray, k: int):
        H = self.hamiltonian_dense(veff)
        w, v = sla.eigh(H, subset_by_index=[0, k - 1], driver="evr")
        return w, v

    # -- SCF ---------------------------------------------------------------
    def kerker(self, r: np.ndarray, q0: float) -> np.ndarray:
        """Kerker preconditioning of a density residual: multiply its Fourier
        components by q^2 / (q^2 + q0^2) (damps long-wavelength charge sloshing)."""
        shape = self.grid.shape_c()
        q2 = np.zeros(shape)
        for ax_c, k in enumerate(reversed(self.grid.n)):
            q = 2.0 * np.pi * np.fft.fftfreq(k, d=self.grid.h)
            sh = [1] * len(shape)
            sh[ax_c] = k
            q2 = q2 + (q ** 2).reshape(sh)
        fr = np.fft.fftn(r.reshape(shape)) * (q2 / (q2 + q0 ** 2))
        return np.fft.ifftn(fr).real.reshape(r.shape)

    def scf(self, tol: float = 1e-12, max_iter: int = 400, beta: float = 0.3,
            history: int = 12, rho0: Optional[np.ndarray] = None, extra_pot=None,
            n_extra: int = 1, q0: float = 0.3, verbose: bool = False) -> GroundState:
        """Self-consistent ground state: Anderson mixing of the density with a
        Kerker-preconditioned residual (the paper uses Anderson mixing, Sec. 4.1).

        extra_pot: an external potential added to V_eff (used for the
        self-consistent response check chi g).
        Converged when max |rho_out - rho_in| <= tol * max(rho).
        """
        n_e = self.n_e
        if rho0 is None:
            rho_in = -self.m.copy()
            # exact neutral start: rescale to the electron count
            rho_in *= (self.f * n_e) / (rho_in.sum() * self.grid.dv)
        else:
            rho_in = rho0.copy()
        X, F = [], []
        res = np.inf
        it = 0
        for it in range(1, max_iter + 1):
            veff = self.veff_of(rho_in)
            if extra_pot is not None:
                veff = veff + extra_pot
            w, v = self.lowest_eigenpairs(veff, n_e + n_extra)
            rho_out = self.density(v[:, :n_e])
            fres = rho_out - rho_in
            res = np.max(np.abs(fres)) / max(np.max(np.abs(rho_out)), 1e-300)
            if verbose:
                print(f"scf {it}: res {res:.3e} gap {w[n_e] - w[n_e - 1]:.6f}")
            if res <= tol:
                break
            X.append(rho_in.copy())
            F.append(fres.copy())
            if len(X) > history:
                X.pop(0)
                F.pop(0)
            if len(X) >= 2:
                dX = np.stack([X[i + 1] - X[i] for i in range(len(X) - 1)], axis=1)
                dF = np.stack([F[i + 1] - F[i] for i in range(len(F) - 1)], axis=1)
                gamma, *_ = np.linalg.lstsq(dF, fres, rcond=None)
                rho_bar = rho_in - dX @ gamma
                f_bar = fres - dF @ gamma
            else:
                rho_bar, f_bar = rho_in, fres
            rho_new = rho_bar + beta * self.kerker(f_bar, q0)
            rho_in = rho_new
        veff = self.veff_of(rho_in)
        if extra_pot is not None:
            veff = veff + extra_pot
        w, v = self.lowest_eigenpairs(veff, n_e + n_extra)
        phi = v[:, :n_e].copy()
        return GroundState(phi=phi, eps=w, veff=veff, rho=self.density(phi), n_e=n_e,
                           scf_iters=it, scf_residual=float(res))

    # -- non-self-consistent inputs for large grids --------------------------
    def superposed_atoms_potential(self, width_factor: float = 1.5) -> np.ndarray:
        """A neutral potential without self-consistency (a Harris-type input):
        V = v_c (rho_at + m), where rho_at puts on every site a Gaussian electron
        cloud of charge Z_I and width width_factor * sigma, so that each
        pseudocharge of Eq. (4.2) is screened by a wider cloud of the same charge.
        The shifted equations of Eq. (3.6) only need some V_eff and its occupied
        eigenpairs; this one has a positive gap for the lattices used here."""
        d = self.grid.dim
        s = width_factor * self.sigma
        D = min_image(self.grid, self.R)
        r2 = np.sum(D * D, axis=2)
        rho_at = (self.Z[None, :] * (2.0 * np.pi * s ** 2) ** (-d / 2.0)
                  * np.exp(-r2 / (2.0 * s ** 2))).sum(axis=1)
        return self.vc(rho_at + self.m)

    def hamiltonian_sparse(self, veff: np.ndarray):
        """H = -1/2 Delta_h + diag(V_eff) as a scipy sparse matrix (CSR)."""
        import scipy.sparse as sp
        mats = []
        for k in self.grid.n:          # periodic 1D second difference, 9 points
            rows, cols, vals = [], [], []
            for sft in range(-4, 5):
                i = np.arange(k)
                rows.append(i)
                cols.append((i + sft) % k)
                vals.append(np.full(k, FD8[abs(sft)]))
            D1 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(k, k))
            mats.append(D1 / self.grid.h ** 2)
        if self.grid.dim == 1:
            lap = mats[0]
        else:   # alpha = ix + nx * iy: x is the fast index
            nx, ny = self.grid.n
            lap = sp.kron(sp.identity(ny), mats[0]) + sp.kron(mats[1], sp.identity(nx))
        return (-0.5 * lap + sp.diags(veff)).tocsr()

    def ground_state_of(self, veff: np.ndarray, n_extra: int = 1, sparse: bool = False) -> GroundState:
        """The lowest N_e + n_extra eigenpairs of H[veff] without SCF (dense eigh,
        or shift-invert Lanczos below the spectrum on the sparse H followed by a
        Rayleigh-Ritz step on the orthonormalised vectors); rho from the
        occupied ones."""
        n_e, k = self.n_e, self.n_e + n_extra
        if not sparse:
            w, v = self.lowest_eigenpairs(veff, k)
        else:
            import scipy.sparse.linalg as spla
            H = self.hamiltonian_sparse(veff)
            w0, v0 = spla.eigsh(H, k=k + 8, sigma=float(veff.min()) - 1.0, which="LM", tol=0.0)
            Qv, _ = np.linalg.qr(v0[:, np.argsort(w0)])
            wr, vr = np.linalg.eigh(Qv.T @ (H @ Qv))
            w, v = wr[:k], Qv @ vr[:, :k]
        phi = v[:, :n_e].copy()
        return GroundState(phi=phi, eps=w, veff=veff.copy(), rho=self.density(phi), n_e=n_e,
                           scf_iters=0, scf_residual=float("nan"))

    # -- energy and forces (Eq. (2.1), Eq. (2.9)) ---------------------------
    def energy(self, gs: GroundState) -> float:
        """E = (f/2) sum_i phi_i^T (-Delta_h) phi_i + (h^d/2)(rho+m)^T v_c (rho+m)
               - (h^d/2) sum_I m_I^T v_c m_I  (pseudocharge form of the ion-ion term)."""
        dv = self.grid.dv
        kin = 0.5 * self.f * np.sum(gs.phi * (-laplacian_apply(self.grid, gs.phi)))
        tot = gs.rho + self.m
        hart = 0.5 * dv * tot @ self.vc(tot)
        self_e = 0.5 * dv * np.sum(self.m_each * self.vc(self.m_each))
        return float(kin + hart - self_e)

    def forces(self, gs: GroundState) -> np.ndarray:
        """Hellmann-Feynman forces F_{I,a} = -h^d (dm_I/dR_{I,a})^T v_c (rho + m - m_I).

        Returned as a vector of length d N_A ordered j = a + d * I.
        """
        dv = self.grid.dv
        d = self.grid.dim
        out = np.empty(self.n_atoms * d)
        base = self.vc(gs.rho + self.m)
        own = self.vc(self.m_each)                  # v_c m_I, N_g x N_A
        for I in range(self.n_atoms):
            pot = base - own[:, I]
            for a in range(d):
                j = a + d * I
                out[j] = -dv * self.dm[:, j] @ pot
        return out

    # -- perturbation vectors and local Hessian terms (Eq. (2.11)) ----------
    def perturbations(self) -> np.ndarray:
        """G = [g_j], g_{I,a} = dV_I/dR_{I,a} = v_c (dm_I / dR_{I,a})  (N_g x d N_A)."""
        return self.vc(self.dm)

    def local_hessian(self, gs: GroundState) -> np.ndarray:
        """Second and third terms of Eq. (2.11) in the pseudocharge form.

        K_{Ia,Jb} = delta_IJ h^d (d2 m_I / dR_a dR_b)^T v_c (rho + m - m_I)
                  + (1 - delta_IJ) h^d (dm_I/dR_a)^T v_c (dm_J/dR_b).
        """
        dv = self.grid.dv
        d = self.grid.dim
        n_p = self.n_atoms * d
        K = dv * (self.dm.T @ self.vc(self.dm))
        base = self.vc(gs.rho + self.m)
        own = self.vc(self.m_each)
        for I in range(self.n_atoms):
            blk = slice(d * I, d * I + d)
            pot = base - own[:, I]
            K[blk, blk] = dv * np.einsum("gab,g->ab", self.d2m[:, I], pot)
        assert K.shape == (n_p, n_p)
        return K


def build_model(cfg, R=None, Z=None, n_e=None) -> Model:
    """Model for a workload configuration (sites from the shared seeded draws)."""
    from workload.seeds import draw_sites
    if R is None:
        R, Z, n_e = draw_sites(cfg)
    grid = Grid(tuple(cfg.n), cfg.h)
    return Model(grid, R, Z, n_e, sigma=cfg.sigma, kappa=cfg.kappa, eps0=cfg.eps0, f=cfg.f)


def frozen_phonon_hessian(model: Model, gs: GroundState, deltas=(1e-2, 5e-3),
                          tol: float = 1e-12) -> np.ndarray:
    """Hessian by central differences of the forces (the frozen-phonon approach
    of Sec. 1), Richardson-extrapolated over two step sizes:
      H_{Ia,Jb} ~ -[F_{Jb}(R + delta e_{Ia}) - F_{Jb}(R - delta e_{Ia})] / (2 delta).
    """
    d = model.grid.dim
    n_p = model.n_atoms * d
    ests = []
    for delta in deltas:
        Hs = np.empty((n_p, n_p))
        for j in range(n_p):
            I, a = divmod(j, d)
            fs = []
            for sgn in (+1.0, -1.0):
                R2 = model.R.copy()
                R2[I, a] += sgn * delta
                m2 = Model(model.grid, R2, model.Z, model.n_e, sigma=model.sigma,
                           kappa=model.kappa, eps0=model.eps0, f=model.f)
                gs2 = m2.scf(tol=tol, rho0=gs.rho)
                fs.append(m2.forces(gs2))
            Hs[j] = -(fs[0] - fs[1]) / (2.0 * delta)
        ests.append(Hs)
    if len(deltas) == 2:
        r = (deltas[0] / deltas[1]) ** 2
        return (r * ests[1] - ests[0]) / (r - 1.0)
    return ests[0]
