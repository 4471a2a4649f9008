"""Pins of the oracle's ACP steps (Alg. 2-4) and of its Krylov solvers (CPU only).

Special cases where ACP must reduce to exact DFPT, interpolation identities,
the interpolative-decomposition error bound, the Sherman-Morrison-Woodbury
identity, and the convergence trend of Table 1.
"""
import numpy as np
import pytest

from oracle import acp as A
from oracle import chi0 as C
from oracle import krylov as K
from oracle.model import build_model, yukawa_dense
from workload.seeds import get_config, draw_sketch


@pytest.fixture(scope="module", params=[1, 11])
def sys_(request):
    cfg = get_config(request.param)
    m = build_model(cfg)
    gs = m.scf(tol=1e-13)
    w, v = C.full_spectrum(m, gs)
    G = m.perturbations()
    om = draw_sketch(cfg, G.shape[1])
    return cfg, m, gs, w, v, G, om


def test_chebyshev_nodes_and_lagrange_weights():
    lo, hi = -1.3, 0.4
    for n_c in (1, 2, 5, 8):
        nodes = A.chebyshev_nodes(lo, hi, n_c)
        # nodes are the images of cos(pi (c - 1/2)/N_c) under x -> (lo+hi)/2 + (lo-hi)/2 x
        t = (nodes - 0.5 * (lo + hi)) / (0.5 * (lo - hi))
        assert np.allclose(t, np.cos(np.pi * (np.arange(1, n_c + 1) - 0.5) / n_c))
        assert np.all((nodes > lo) & (nodes < hi))
        if n_c > 1:
            L = A.lagrange_weights(nodes, nodes)
            assert np.allclose(L, np.eye(n_c), atol=1e-13)
            x = np.linspace(lo, hi, 17)
            L = A.lagrange_weights(nodes, x)
            assert np.allclose(L.sum(axis=0), 1.0, atol=1e-13)
            # exact on polynomials of degree < N_c
            p = lambda e: 0.3 * e ** (n_c - 1) - e + 2.0
            assert np.allclose(p(nodes) @ L, p(x), atol=1e-12)


def test_chebyshev_error_bound_for_resolvent():
    """Interpolating 1/(lam - e) on [e_1, e_N] at N_c Chebyshev points obeys the
    Bernstein-ellipse bound 4 M rho'^{-(N_c - 1)} / (rho' - 1) (Trefethen, ATAP,
    Thm 8.2).  In the normalised variable the pole sits at alpha = 1 + 2 gap/width,
    so any rho' < alpha + sqrt(alpha^2 - 1) works with
    M = 1 / (half_width * (alpha - (rho' + 1/rho') / 2))."""
    lo, hi, gap = -1.0, -0.2, 0.3
    lam = hi + gap
    x = np.linspace(lo, hi, 101)
    hw = 0.5 * (hi - lo)
    alpha = 1 + gap / hw
    rho = alpha + np.sqrt(alpha ** 2 - 1)
    rho_p = 0.5 * (1.0 + rho)
    M = 1.0 / (hw * (alpha - 0.5 * (rho_p + 1.0 / rho_p)))
    for n_c in (4, 8, 12):
        nodes = A.chebyshev_nodes(lo, hi, n_c)
        L = A.lagrange_weights(nodes, x)
        err = np.abs((1.0 / (lam - nodes)) @ L - 1.0 / (lam - x)).max()
        assert err <= 4 * M * rho_p ** (-(n_c - 1)) / (rho_p - 1)
        assert err > 1e-3 * 4 * M * rho ** (-(n_c - 1)) / (rho - 1)  # and not trivially small


def test_isdf_interpolates_and_matches_forced_selection(sys_):
    cfg, m, gs, w, v, G, om = sys_
    dec = A.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    Mt = A.sketched_rows(gs.phi, G, om)
    assert np.array_equal(dec.xi[dec.sel], np.eye(cfg.n_mu))
    assert len(np.unique(dec.sel)) == cfg.n_mu
    # ID error of the order of the discarded part of R (Alg. 2 step 4)
    r22 = np.sqrt(np.sum(dec.rdiag[cfg.n_mu:] ** 2))
    res = A.id_residual(gs.phi, G, om, dec)
    assert res <= 10 * np.sqrt(Mt.shape[1]) * max(r22, 1e-14 * np.linalg.norm(Mt))
    # the same selection through the least-squares definition gives the same Xi
    dec2 = A.isdf_forced(gs.phi, G, om, dec.sel)
    assert np.abs(dec.xi - dec2.xi).max() < 1e-8 * np.abs(dec.xi).max()


def test_isdf_pivots_are_greedy_maxima(sys_):
    """Column-pivoted QR: pivot k is the row of M~ with the largest norm after
    projecting out the rows already chosen (brute force)."""
    cfg, m, gs, w, v, G, om = sys_
    dec = A.isdf_qrcp(gs.phi, G, om, 8)
    Mt = A.sketched_rows(gs.phi, G, om)
    chosen = []
    for k in range(8):
        if chosen:
            B = Mt[chosen].T
            Qb, _ = np.linalg.qr(B)
            Rm = Mt - (Mt @ Qb) @ Qb.T
        else:
            Rm = Mt
        nrm = np.sum(Rm * Rm, axis=1)
        assert nrm[dec.sel[k]] >= (1 - 1e-10) * nrm.max()
        chosen.append(dec.sel[k])


def test_w_matches_unsimplified_definition(sys_):
    """Eq. (3.7) assembled as written: W_mu = 2f/h^d sum_i phi_i o (sum_c zeta~_{c mu} L_c(eps_i)) phi_i(r_mu)."""
    cfg, m, gs, w, v, G, om = sys_
    dec = A.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    nodes, L = A.shifts_and_weights(gs.eps[:gs.n_e], cfg.n_cheb)
    R = A.rhs(gs.phi, dec.xi)
    solver = A.ExactShiftedSolver(w, v, gs.n_e)
    Z = A.solve_compressed(solver, nodes, R)
    W = A.assemble_w(gs.phi, L, dec.sel, Z, m.f, m.grid.dv)
    W2 = np.zeros_like(W)
    for mu in range(cfg.n_mu):
        for i in range(gs.n_e):
            zi = sum(Z[c][:, mu] * L[c, i] for c in range(len(nodes)))
            W2[:, mu] += gs.phi[:, i] * zi * gs.phi[dec.sel[mu], i]
    W2 *= 2 * m.f / m.grid.dv
    assert np.abs(W - W2).max() < 1e-12 * np.abs(W).max()


def test_acp_is_exact_dfpt_with_identity_isdf_and_occupied_nodes(sys_):
    """With every grid point selected (Xi = I) and the occupied eigenvalues as
    nodes, chi0~ = chi0 and Alg. 4 reproduces chi G after one update."""
    cfg, m, gs, w, v, G, om = sys_
    n_g = m.grid.n_grid
    X0 = C.chi0_sos_matrix(m, w, v, gs.n_e)
    Vc = yukawa_dense(m.grid, m.kappa, m.eps0)
    U_exact = C.dyson_dense(X0, Vc, G)
    solver = A.ExactShiftedSolver(w, v, gs.n_e)
    sel = np.arange(n_g)
    res = A.acp_dyson(gs.phi, gs.eps[:gs.n_e], G, om, cfg.n_cheb, n_g, solver, vc=m.vc,
                      vc_inv=m.vc_inv, f=m.f, dv=m.grid.dv, k_max=2, sel_hist=[sel, sel],
                      node_mode="occupied")
    assert np.abs(res.W_hist[0] - X0).max() < 1e-11 * np.abs(X0).max()
    assert np.linalg.norm(res.U - U_exact) < 1e-10 * np.linalg.norm(U_exact)
    # chi0~ X = W X(Pi, :) is then chi0 X
    Y = A.chi0_tilde_apply(res.W_hist[0], sel, G)
    assert np.abs(Y - X0 @ G).max() < 1e-11 * np.abs(X0 @ G).max()


def test_smw_update_equals_dense_inverse(sys_):
    """Eq. (3.13): B + W (I - Pi^T v W)^{-1} Pi^T v B = (I - W Pi^T v)^{-1} B."""
    cfg, m, gs, w, v, G, om = sys_
    solver = A.ExactShiftedSolver(w, v, gs.n_e)
    comp = A.compress(gs.phi, gs.eps[:gs.n_e], G, om, cfg.n_cheb, cfg.n_mu, solver, m.f, m.grid.dv)
    Vc = yukawa_dense(m.grid, m.kappa, m.eps0)
    B = m.vc_inv(G)
    dense = A.smw_dense_reference(comp.W, comp.sel, Vc, B)
    V = m.vc(comp.W)
    S = np.linalg.solve(np.eye(cfg.n_mu) - V[comp.sel], G[comp.sel])
    smw = B + comp.W @ S
    assert np.abs(dense - smw).max() < 1e-9 * np.abs(dense).max()


def test_acp_error_decreases_with_rank():
    """Table 1 trend: at fixed N_c the error of chi G decreases with N_mu."""
    cfg = get_config(11)
    m = build_model(cfg)
    gs = m.scf(tol=1e-13)
    w, v = C.full_spectrum(m, gs)
    G = m.perturbations()
    om = draw_sketch(cfg, G.shape[1])
    X0 = C.chi0_sos_matrix(m, w, v, gs.n_e)
    U = C.dyson_dense(X0, yukawa_dense(m.grid, m.kappa, m.eps0), G)
    solver = A.ExactShiftedSolver(w, v, gs.n_e)
    errs = []
    for l in (2, 4, 6):
        res = A.acp_dyson(gs.phi, gs.eps[:gs.n_e], G, om, 10, l * gs.n_e, solver, vc=m.vc,
                          vc_inv=m.vc_inv, f=m.f, dv=m.grid.dv, k_max=4)
        errs.append(np.linalg.norm(res.U - U) / np.linalg.norm(U))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


@pytest.mark.parametrize("solver", ["cg", "minres"])
def test_krylov_solvers_match_exact(sys_, solver):
    cfg, m, gs, w, v, G, om = sys_
    dec = A.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    nodes, _ = A.shifts_and_weights(gs.eps[:gs.n_e], cfg.n_cheb)
    R = A.rhs(gs.phi, dec.xi)
    shifts = np.repeat(nodes, R.shape[1])
    B = np.tile(R, (1, len(nodes)))
    op = K.make_operator(m, gs.veff, gs.phi, shifts)
    fn = K.cg if solver == "cg" else K.minres
    x, it, _ = fn(op, B, 1e-11)
    assert K.true_residual(op, x, B).max() < 2e-11
    ex = np.concatenate([A.ExactShiftedSolver(w, v, gs.n_e)(s, R) for s in nodes], axis=1)
    assert np.abs(x - ex).max() < 1e-8 * np.abs(ex).max()
    # the dense factorisation of Q(H - s)Q + Phi Phi^T gives the same solutions
    dense = A.DenseShiftedSolver(m.hamiltonian_dense(gs.veff), gs.phi)
    ex2 = np.concatenate([dense(s, R) for s in nodes], axis=1)
    assert np.abs(ex2 - ex).max() < 1e-9 * np.abs(ex).max()


def test_isdf_rank_rule_on_prescribed_pivots():
    """Alg. 2 step 3: the rank is the number of pivots whose |R_kk| is at least
    tol |R_11|.  Pin: with one orbital equal to 1 everywhere and Omega = I, the
    sketched matrix M~ is G itself; G has nonzero rows only at five grid points,
    each a multiple of a different unit vector, so the pivoted QR takes those
    rows in decreasing size with |R_kk| equal to the sizes (orthogonal rows).
    An off-by-one in the rule, or a rule on the wrong end of the threshold,
    changes the rank or the selected points."""
    n_g, n_p = 48, 6
    pts = np.array([17, 3, 40, 8, 25])
    size = np.array([1e-2, 1.0, 1e-4, 1e-1, 1e-3])
    G = np.zeros((n_g, n_p))
    G[pts, np.arange(5)] = size
    phi = np.ones((n_g, 1))
    om = np.eye(n_p)
    order = pts[np.argsort(-size)]              # 3, 8, 17, 25, 40
    for tol, rank in ((5e-3, 3), (5e-2, 2), (0.5, 1), (5e-4, 4), (5e-5, 5)):
        dec = A.isdf_qrcp(phi, G, om, 5, tol=tol)
        assert len(dec.sel) == rank, (tol, len(dec.sel))
        assert np.array_equal(dec.sel, order[:rank])
        assert np.allclose(dec.rdiag[:5], np.sort(size)[::-1], rtol=1e-12, atol=0)
    # the fixed rank caps the rule
    dec = A.isdf_qrcp(phi, G, om, 2, tol=5e-4)
    assert np.array_equal(dec.sel, order[:2])
    # tol = 0 keeps the fixed rank even past the numerical rank of the sketch
    assert len(A.isdf_qrcp(phi, G, om, 5).sel) == 5


def test_dyson_stop_rule(sys_):
    """Alg. 4 stops after the first compression whose relative change
    ||U^k - U^{k-1}||_F / ||U^k||_F is at most delta.  Pin: with every grid
    point selected and the occupied eigenvalues as nodes the compression is
    exact, so U^1 is already chi G (the change of the first iteration, from
    U^0 = 0, is exactly 1) and U^2 repeats it to rounding.  Hence delta = 1e-9
    stops after exactly 2 compressions, delta >= 1 after 1, and delta = 0 runs
    k_max."""
    cfg, m, gs, w, v, G, om = sys_
    n_g = m.grid.n_grid
    solver = A.ExactShiftedSolver(w, v, gs.n_e)
    sel = np.arange(n_g)
    common = dict(vc=m.vc, vc_inv=m.vc_inv, f=m.f, dv=m.grid.dv, sel_hist=[sel] * 3,
                  node_mode="occupied")
    args = (gs.phi, gs.eps[:gs.n_e], G, om, cfg.n_cheb, n_g, solver)
    r = A.acp_dyson(*args, k_max=3, delta=1e-9, **common)
    assert r.iters == 2 and len(r.changes) == 2
    assert r.changes[0] == 1.0 and r.changes[1] < 1e-9
    assert A.acp_dyson(*args, k_max=3, delta=1.0, **common).iters == 1
    assert A.acp_dyson(*args, k_max=3, delta=0.0, **common).iters == 3


def test_projected_spectral_solver(sys_):
    """The eigenpairs of Q H Q + c P give the solution of Q (H - s) Q z = b for
    any orthonormal Phi: equal to the dense factorisation (random Phi), to the
    exact solver (Phi = occupied eigenvectors), and z solves the equation."""
    cfg, m, gs, w, v, G, om = sys_
    H = m.hamiltonian_dense(gs.veff)
    rng = np.random.default_rng(2)
    n = H.shape[0]
    phi, _ = np.linalg.qr(rng.standard_normal((n, 12)))
    b = A.project_q(phi, rng.standard_normal((n, 3)))
    s = float(np.linalg.eigvalsh(H)[0]) - 0.5
    z = A.ProjectedSpectralSolver(H, phi)(s, b)
    zd = A.DenseShiftedSolver(H, phi)(s, b)
    assert np.abs(z - zd).max() < 1e-10 * np.abs(zd).max()
    Q = np.eye(n) - phi @ phi.T
    assert np.abs(Q @ (H - s * np.eye(n)) @ Q @ z - b).max() < 1e-10 * np.abs(b).max()
    R = A.project_q(gs.phi, rng.standard_normal((n, 3)))
    s2 = float(gs.eps[0])
    ze = A.ExactShiftedSolver(w, v, gs.n_e)(s2, R)
    zp = A.ProjectedSpectralSolver(H, gs.phi)(s2, R)
    assert np.abs(zp - ze).max() < 1e-9 * np.abs(ze).max()
