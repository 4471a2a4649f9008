"""Pins of the oracle's discrete model against closed forms, the mathematics and
the numbers printed in the paper (CPU only)."""
import json
import os

import numpy as np
import pytest
from scipy.special import erfc

from oracle.model import (FD8, Grid, Model, build_model, fd_symbol_1d, laplacian_apply,
                          yukawa_apply, yukawa_inverse_apply, pseudocharges)
from workload.seeds import get_config, draw_sites

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- finite-difference Laplacian --------------------------------------------
def test_fd8_coefficients_taylor_conditions():
    """Central 8th-order second derivative: sum c_s s^0 = 0, sum c_s s^2 = 1,
    sum c_s s^{2j} = 0 for j = 2, 3, 4 (sum over s = -4..4)."""
    s = np.arange(-4, 5)
    c = FD8[np.abs(s)]
    assert abs(c.sum()) < 1e-15
    assert abs((c * s ** 2).sum() - 2.0) < 1e-14  # (1/2) * 2! for the s^2 Taylor term
    for j in (2, 3, 4):
        assert abs((c * s ** (2 * j)).sum()) < 1e-11


@pytest.mark.parametrize("n,dim", [(48, 1), (40, 2)])
def test_plane_wave_is_eigenvector_with_fd_symbol(n, dim):
    h = 0.37
    g = Grid((n,) * dim if dim == 2 else (n,), h)
    X = g.coords()
    k = np.array([3, 5][:dim])
    theta = 2 * np.pi * k / n
    u = np.cos(X @ (theta / h))
    lam = sum(fd_symbol_1d(n, h)[kk] for kk in k)
    assert np.allclose(-laplacian_apply(g, u), lam * u, rtol=0, atol=1e-12 * lam)
    # closed form of the symbol against the stencil sum
    closed = (2 * np.sum(FD8[1:] * (1 - np.cos(np.arange(1, 5) * theta[0])))) / h ** 2
    assert abs(fd_symbol_1d(n, h)[k[0]] - closed) < 1e-12 * closed


def test_laplacian_eighth_order_convergence():
    errs = []
    for n in (32, 64):
        L = 2 * np.pi
        g = Grid((n,), L / n)
        x = g.coords()[:, 0]
        u = np.exp(np.sin(x))
        exact = np.exp(np.sin(x)) * (np.cos(x) ** 2 - np.sin(x))
        errs.append(np.abs(laplacian_apply(g, u) - exact).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > 7.5


# --- Yukawa operator ----------------------------------------------------------
@pytest.mark.parametrize("n", [(64,), (24, 20)])
def test_yukawa_inverse_pair(n):
    g = Grid(n, 0.5)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((g.n_grid, 3))
    y = yukawa_apply(g, 0.05, 2.0, x)
    assert np.allclose(yukawa_inverse_apply(g, 0.05, 2.0, y), x, atol=1e-11)


def test_yukawa_continuum_kernel_1d():
    """Eq. (4.3): K(x) = 2 pi exp(-kappa |x|) / (kappa eps0).  The discrete v_c of a
    Gaussian of width s equals the periodised convolution of K with it, whose
    closed form uses erfc."""
    kappa, eps0, s, L, n = 0.05, 2.0, 2.0, 80.0, 640
    g = Grid((n,), L / n)
    x = g.coords()[:, 0]
    x0 = 37.3
    d = x - x0
    d = d - L * np.round(d / L)
    rho = np.exp(-d ** 2 / (2 * s ** 2)) / np.sqrt(2 * np.pi * s ** 2)
    num = yukawa_apply(g, kappa, eps0, rho)
    ref = np.zeros_like(x)
    for img in range(-60, 61):
        t = d + img * L
        a = np.exp(kappa ** 2 * s ** 2 / 2) * 0.5 * (
            np.exp(-kappa * t) * erfc((kappa * s ** 2 - t) / (s * np.sqrt(2)))
            + np.exp(kappa * t) * erfc((kappa * s ** 2 + t) / (s * np.sqrt(2))))
        ref += a
    ref *= 2 * np.pi / (kappa * eps0)
    assert np.abs(num - ref).max() < 1e-8 * np.abs(ref).max()


# --- pseudocharges --------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2])
def test_pseudocharge_normalisation_and_derivatives(dim):
    n = (160,) if dim == 1 else (48, 48)
    g = Grid(n, 0.25)
    R = np.array([[7.3, 5.1][:dim], [31.9, 9.7][:dim]])
    Z = np.array([2.0, 1.7])
    m, dm, d2m = pseudocharges(g, R, Z, 1.0)
    assert np.allclose(m.sum(axis=0) * g.dv, -Z, rtol=1e-12)
    eps = 1e-5
    for I in range(2):
        for a in range(dim):
            Rp, Rm = R.copy(), R.copy()
            Rp[I, a] += eps
            Rm[I, a] -= eps
            fd = (pseudocharges(g, Rp, Z, 1.0)[0][:, I] - pseudocharges(g, Rm, Z, 1.0)[0][:, I]) / (2 * eps)
            assert np.allclose(dm[:, a + dim * I], fd, atol=1e-8)
            fd2 = (pseudocharges(g, Rp, Z, 1.0)[1][:, a + dim * I]
                   - pseudocharges(g, Rm, Z, 1.0)[1][:, a + dim * I]) / (2 * eps)
            assert np.allclose(d2m[:, I, a, a], fd2, atol=1e-7)


# --- ground state ------------------------------------------------------------
def _paper_model(n_atoms, eps0, h=0.1, a=2.4):
    n = int(round(n_atoms * a / h))
    g = Grid((n,), n_atoms * a / n)
    R = ((np.arange(n_atoms) + 0.5) * a).reshape(-1, 1)
    return Model(g, R, np.ones(n_atoms), n_atoms, sigma=0.3, kappa=0.1, eps0=eps0, f=1.0)


@pytest.mark.parametrize("case", [0, 1])
def test_paper_1d_ground_state_golden(case):
    """Gap and density range of the paper's 60-atom 1D insulator/semiconductor."""
    gold = json.load(open(os.path.join(GOLDEN, "paper_1d_ground_state.json")))
    c = gold["cases"][case]
    m = _paper_model(gold["model"]["n_atoms"], c["eps0"])
    gs = m.scf(tol=1e-10)
    half_ulp = 0.5 * 10.0 ** -c["printed_digits"]
    assert abs(gs.gap - c["gap"]) <= half_ulp
    assert abs(gs.rho.min() - c["rho_min"]) <= half_ulp
    assert abs(gs.rho.max() - c["rho_max"]) <= half_ulp


@pytest.fixture(scope="module")
def cfg1_gs():
    m = build_model(get_config(1))
    return m, m.scf(tol=1e-13)


def test_ground_state_is_eigen_and_self_consistent(cfg1_gs):
    m, gs = cfg1_gs
    H = m.hamiltonian_dense(gs.veff)
    phi = gs.phi
    assert np.abs(H @ phi - phi * gs.eps[:gs.n_e]).max() < 1e-11
    assert np.abs(phi.T @ phi - np.eye(gs.n_e)).max() < 1e-13
    assert gs.gap > 0.1
    # neutrality and self-consistency V = v_c(rho + m)
    assert abs((gs.rho + m.m).sum() * m.grid.dv) < 1e-10
    assert np.abs(gs.veff - m.vc(gs.rho + m.m)).max() < 1e-9


def test_forces_match_energy_derivative():
    """Eq. (2.9) (Hellmann-Feynman) against a central difference of the total energy."""
    cfg = get_config(11)
    m = build_model(cfg)
    gs = m.scf(tol=1e-13)
    F = m.forces(gs)
    d = 1e-4
    for j in (0, 5):
        E = []
        for sgn in (1, -1):
            R2 = m.R.copy()
            R2[j, 0] += sgn * d
            m2 = Model(m.grid, R2, m.Z, m.n_e, sigma=m.sigma, kappa=m.kappa, eps0=m.eps0, f=m.f)
            E.append(m2.energy(m2.scf(tol=1e-13, rho0=gs.rho)))
        fd = -(E[0] - E[1]) / (2 * d)
        assert abs(F[j] - fd) < 1e-7 * max(1.0, np.abs(F).max())


def test_sites_are_deterministic_and_neutral():
    for cid in (1, 2, 3):
        cfg = get_config(cid)
        R1, Z1, ne1 = draw_sites(cfg)
        R2, Z2, ne2 = draw_sites(cfg)
        assert np.array_equal(R1, R2) and np.array_equal(Z1, Z2)
        assert abs(Z1.sum() - cfg.f * ne1) < 1e-10
        assert R1.shape == (int(np.prod(cfg.sites)), cfg.dim)


def test_sparse_hamiltonian_and_non_scf_ground_state():
    """The sparse H equals the stencil apply (plane waves are eigenvectors with
    the closed-form symbol plus the constant potential); the shift-invert
    eigenpairs equal the dense ones; the superposed-atom potential comes from a
    neutral charge (rho_at + m integrates to zero) and has a positive gap."""
    from workload.seeds import small_config
    cfg = small_config(901, 2, 3, 10, a=6.0, sigma=0.8, jitter=0.05)
    m = build_model(cfg)
    n = m.grid.n_grid
    H0 = m.hamiltonian_sparse(np.full(n, 0.25))
    kx, ky = 3, 7
    X = m.grid.coords()
    L = np.array(m.grid.box)
    pw = np.cos(2 * np.pi * (kx * X[:, 0] / L[0] + ky * X[:, 1] / L[1]))
    from oracle.model import fd_symbol_1d
    lam = 0.5 * (fd_symbol_1d(m.grid.n[0], m.grid.h)[kx] + fd_symbol_1d(m.grid.n[1], m.grid.h)[ky]) + 0.25
    assert np.abs(H0 @ pw - lam * pw).max() < 1e-12 * lam
    V = m.superposed_atoms_potential()
    x = np.random.default_rng(1).standard_normal(n)
    assert np.abs(m.hamiltonian_sparse(V) @ x - m.hamiltonian_apply(V, x)).max() < 1e-12
    # V = v_c q with q neutral: v_c^{-1} V integrates to zero
    assert abs(m.vc_inv(V).sum()) * m.grid.dv < 1e-10
    gd = m.ground_state_of(V)
    gsp = m.ground_state_of(V, sparse=True)
    assert gd.gap > 0.1
    assert np.abs(gd.eps - gsp.eps).max() < 1e-11
    Hd = m.hamiltonian_dense(V)
    assert np.abs(Hd @ gsp.phi - gsp.phi * gsp.eps[:m.n_e]).max() < 1e-11
    assert np.abs(gsp.phi.T @ gsp.phi - np.eye(m.n_e)).max() < 1e-13
