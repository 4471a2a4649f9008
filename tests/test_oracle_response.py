"""Pins of the oracle's exact response: chi0, chi, the Hessian (CPU only).

Two independent formulas for chi0 (sum over states and the Sternheimer form of
Alg. 1), brute-force finite-difference density responses, the frozen-phonon
Hessian, symmetry, semi-definiteness and the acoustic sum rule.
"""
import numpy as np
import pytest

from oracle import chi0 as C
from oracle.model import Model, build_model, frozen_phonon_hessian, yukawa_dense
from workload.seeds import get_config


@pytest.fixture(scope="module", params=[11, 1])
def system(request):
    cfg = get_config(request.param)
    m = build_model(cfg)
    gs = m.scf(tol=1e-13)
    w, v = C.full_spectrum(m, gs)
    X0 = C.chi0_sos_matrix(m, w, v, gs.n_e)
    G = m.perturbations()
    Vc = yukawa_dense(m.grid, m.kappa, m.eps0)
    return cfg, m, gs, w, v, X0, G, Vc


def test_sos_equals_sternheimer_alg1(system):
    _, m, gs, w, v, X0, G, _ = system
    a = X0 @ G
    b = C.chi0_apply_sternheimer(m, gs, G)
    assert np.abs(a - b).max() < 1e-11 * np.abs(a).max()
    c = C.chi0_apply_sos(m, w, v, gs.n_e, G)
    assert np.abs(a - c).max() < 1e-12 * np.abs(a).max()


def test_chi0_symmetric_negative_semidefinite_annihilates_constants(system):
    _, m, gs, w, v, X0, G, _ = system
    s = np.abs(X0).max()
    assert np.abs(X0 - X0.T).max() < 1e-13 * s
    assert np.linalg.eigvalsh(X0).max() < 1e-12 * s
    one = np.ones(X0.shape[0])
    assert np.abs(X0 @ one).max() < 1e-12 * s


def test_chi0_equals_brute_force_density_response(system):
    """chi0 g = d rho / d V along g: central difference of the non-self-consistent
    density of H[V_eff + t g] (exact to O(t^2))."""
    _, m, gs, w, v, X0, G, _ = system
    g = G[:, 0] / np.abs(G[:, 0]).max()
    t = 1e-4
    rhos = []
    for sgn in (1, -1):
        ww, vv = m.lowest_eigenpairs(gs.veff + sgn * t * g, gs.n_e)
        rhos.append(m.density(vv))
    fd = (rhos[0] - rhos[1]) / (2 * t)
    ref = X0 @ g
    assert np.abs(fd - ref).max() < 1e-5 * np.abs(ref).max()


def test_chi_equals_self_consistent_response(system):
    """chi g (Eq. (2.14)) against the change of the SCF density under an external
    potential t g (central difference)."""
    _, m, gs, w, v, X0, G, Vc = system
    g = G[:, 1] / np.abs(G[:, 1]).max()
    U = C.dyson_dense(X0, Vc, g[:, None])[:, 0]
    t = 1e-4
    rhos = []
    for sgn in (1, -1):
        gs2 = m.scf(tol=1e-13, rho0=gs.rho, extra_pot=sgn * t * g)
        rhos.append(gs2.rho)
    fd = (rhos[0] - rhos[1]) / (2 * t)
    assert np.abs(fd - U).max() < 1e-5 * np.abs(U).max()


def test_dyson_dense_equals_neumann_when_contractive():
    """Eq. (2.16) converges to Eq. (2.14) when the spectral radius of chi0 v_c < 1;
    a weak Yukawa prefactor (large eps0) makes it contractive."""
    cfg = get_config(11)
    m = build_model(cfg)
    m.eps0 = 40.0
    gs = m.scf(tol=1e-12)
    w, v = C.full_spectrum(m, gs)
    X0 = C.chi0_sos_matrix(m, w, v, gs.n_e)
    Vc = yukawa_dense(m.grid, m.kappa, m.eps0)
    rho_sr = np.abs(np.linalg.eigvals(X0 @ Vc)).max()
    assert rho_sr < 0.9
    G = m.perturbations()
    a = C.dyson_dense(X0, Vc, G)
    b = C.dyson_neumann(X0, Vc, G, 400)
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()


def test_hessian_symmetric_and_acoustic_sum_rule(system):
    _, m, gs, w, v, X0, G, Vc = system
    U = C.dyson_dense(X0, Vc, G)
    H = C.hessian_exact(m, gs, U, G)
    scale = np.abs(m.local_hessian(gs)).max()   # size of the cancelling terms
    assert np.abs(H - H.T).max() < 1e-9 * scale
    assert np.abs(H.sum(axis=1)).max() < 1e-9 * scale


def test_hessian_matches_frozen_phonon():
    """Eq. (2.11) against finite differences of the Hellmann-Feynman forces (the
    frozen-phonon approach of Sec. 1), Richardson-extrapolated."""
    cfg = get_config(11)
    m = build_model(cfg)
    # a shorter chain keeps the 4 N_A SCF runs cheap
    m = Model(m.grid.__class__((96,), m.grid.h), m.R[:4], m.Z[:4], 4, sigma=m.sigma,
              kappa=m.kappa, eps0=m.eps0, f=m.f)
    gs = m.scf(tol=1e-13)
    w, v = C.full_spectrum(m, gs)
    X0 = C.chi0_sos_matrix(m, w, v, gs.n_e)
    G = m.perturbations()
    U = C.dyson_dense(X0, yukawa_dense(m.grid, m.kappa, m.eps0), G)
    H = C.hessian_exact(m, gs, U, G)
    Hfd = frozen_phonon_hessian(m, gs, tol=1e-13)
    assert np.abs(H - Hfd).max() < 1e-6 * np.abs(H).max()
    D, lam = C.dynamical_matrix(H, np.ones(4), 1)
    assert abs(lam[0]) < 1e-9 * lam[-1]          # one acoustic mode at zero
    assert lam[1] > 0                             # stable chain


def test_dynamical_matrix_with_masses_is_generalised_eigenproblem():
    """D = M^{-1/2} Hess M^{-1/2} has the eigenvalues of Hess u = omega^2 M u
    (a library routine for the symmetric-definite generalised problem)."""
    import scipy.linalg as sla
    rng = np.random.default_rng(4)
    d, n_a = 2, 5
    H = rng.standard_normal((d * n_a, d * n_a))
    masses = rng.uniform(1.0, 30.0, n_a)
    D, lam = C.dynamical_matrix(H, masses, d)
    Hs = 0.5 * (H + H.T)
    ref = sla.eigh(Hs, np.diag(np.repeat(masses, d)), eigvals_only=True)
    assert np.allclose(lam, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(D, D.T)


def test_phonon_dos_normalisation_and_closed_forms():
    """The smeared phonon spectrum integrates to n / (d N_A); one mode at
    omega^2 = 4 is the Gaussian around 2; negative omega^2 gives negative
    frequencies; the sum over modes is linear."""
    sigma = 0.08
    w = np.linspace(-3.0, 6.0, 9001)
    lam = np.array([0.0, 0.25, 1.0, 4.0, 4.0, 9.0])
    rho = C.phonon_dos(lam, 6, sigma, w)
    assert abs(np.trapezoid(rho, w) - 1.0) < 1e-10
    one = C.phonon_dos(np.array([4.0]), 2, sigma, w)
    peak = 1.0 / (np.sqrt(2 * np.pi) * sigma) / 2
    assert abs(one[np.argmin(np.abs(w - 2.0))] - peak) < 1e-12
    assert abs(one[np.argmin(np.abs(w - 2.0 - sigma))] - peak * np.exp(-0.5)) < 1e-12
    neg = C.phonon_dos(np.array([-1e-4]), 1, sigma, w)
    assert abs(w[np.argmax(neg)] + 1e-2) < 2e-3
    parts = sum(C.phonon_dos(lam[i:i + 1], 6, sigma, w) for i in range(6))
    assert np.allclose(parts, rho, rtol=0, atol=1e-14)

