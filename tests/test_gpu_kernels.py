"""GPU parity of the hot-path building blocks against the CPU oracle:
the stencil H - s (K1), v_c and v_c^{-1}, and the batched projected shifted
solves (CG and MINRES) through the C ABI."""
import numpy as np
import pytest

from tests.gpu_common import make_ctx, require_gpu, system, to_dev, to_host
from oracle import acp as OA
from oracle import krylov as OK
from oracle.model import Grid, yukawa_apply, yukawa_inverse_apply

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("cid", [1, 11])
def test_apply_h_matches_oracle(cid):
    cfg, m, gs, w, v, G, om, K = system(cid)
    ctx = make_ctx(cid)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((m.grid.n_grid, 37))
    sh = rng.uniform(-1, 0, 37)
    Y = to_host(ctx.apply_h(to_dev(X), sh))
    ref = m.hamiltonian_apply(gs.veff, X) - X * sh[None, :]
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("shape", [(96, 80), (150, 41), (68, 20), (67, 19)])
def test_apply_h_2d_tiles_wrap(shape):
    """2D grids ragged against the 64 x 16 stencil tiles: from 68 x 20 up the
    halo wraps with one add or subtract, below it by the remainder (67 x 19)."""
    from paper_1605_08021_amd import acp
    g = Grid(shape, 0.5)
    rng = np.random.default_rng(8)
    V = rng.standard_normal(g.n_grid)
    phi, _ = np.linalg.qr(rng.standard_normal((g.n_grid, 5)))
    ctx = acp.Context(dict(dim=2, n=shape, h=0.5, kappa=0.05, eps0=1.0, occ=2.0),
                      dict(n_cheb=2, n_mu=8, sketch_r=2), to_dev(phi), np.linspace(-1, -0.5, 5),
                      to_dev(V))
    X = rng.standard_normal((g.n_grid, 7))
    sh = rng.standard_normal(7)
    Y = to_host(ctx.apply_h(to_dev(X), sh))
    from oracle.model import laplacian_apply
    ref = -0.5 * laplacian_apply(g, X) + V[:, None] * X - sh[None, :] * X
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


def test_apply_h_2d_ragged():
    """2D grid with sides that are not multiples of any tile size."""
    from paper_1605_08021_amd import acp
    g = Grid((27, 22), 0.5)
    rng = np.random.default_rng(7)
    V = rng.standard_normal(g.n_grid)
    phi, _ = np.linalg.qr(rng.standard_normal((g.n_grid, 5)))
    ctx = acp.Context(dict(dim=2, n=(27, 22), h=0.5, kappa=0.05, eps0=1.0, occ=2.0),
                      dict(n_cheb=2, n_mu=8, sketch_r=2), to_dev(phi), np.linspace(-1, -0.5, 5),
                      to_dev(V))
    X = rng.standard_normal((g.n_grid, 19))
    Y = to_host(ctx.apply_h(to_dev(X)))
    from oracle.model import laplacian_apply
    ref = -0.5 * laplacian_apply(g, X) + V[:, None] * X
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    Yv = to_host(ctx.apply_vc(to_dev(X)))
    refv = yukawa_apply(g, 0.05, 1.0, X)
    assert np.abs(Yv - refv).max() <= 1e-12 * np.abs(refv).max()
    Yi = to_host(ctx.apply_vc_inv(to_dev(X)))
    refi = yukawa_inverse_apply(g, 0.05, 1.0, X)
    assert np.abs(Yi - refi).max() <= 1e-13 * np.abs(refi).max()
    ctx.close()


@pytest.mark.parametrize("cid", [1, 11])
def test_yukawa_pair_matches_oracle(cid):
    cfg, m, gs, w, v, G, om, K = system(cid)
    ctx = make_ctx(cid)
    Y = to_host(ctx.apply_vc(to_dev(G)))
    ref = m.vc(G)
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()
    B = to_host(ctx.apply_vc_inv(to_dev(G)))
    refb = m.vc_inv(G)
    assert np.abs(B - refb).max() <= 1e-13 * np.abs(refb).max()
    ctx.close()


def _rhs_batch(cid, n_cols=None):
    cfg, m, gs, w, v, G, om, K = system(cid)
    dec = OA.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    nodes, _ = OA.shifts_and_weights(gs.eps[:gs.n_e], cfg.n_cheb)
    R = OA.rhs(gs.phi, dec.xi)
    shifts = np.repeat(nodes, R.shape[1])
    B = np.tile(R, (1, len(nodes)))
    if n_cols is not None:
        B, shifts = B[:, :n_cols], shifts[:n_cols]
    exact = np.concatenate([OA.ExactShiftedSolver(w, v, gs.n_e)(s, R) for s in nodes], axis=1)
    if n_cols is not None:
        exact = exact[:, :n_cols]
    return m, gs, B, shifts, exact


@pytest.mark.parametrize("cid", [1, 11])
@pytest.mark.parametrize("solver", [0, 1])
def test_sternheimer_matches_exact_solution(cid, solver):
    m, gs, B, shifts, exact = _rhs_batch(cid, n_cols=None)
    # a ragged batch: not a multiple of the 16-system tile
    B, shifts, exact = B[:, :-5], shifts[:-5], exact[:, :-5]
    ctx = make_ctx(cid, solver=solver, tol=1e-12)
    X, iters, _ = ctx.sternheimer(shifts, to_dev(B))
    X = to_host(X)
    rel = np.abs(X - exact).max() / np.abs(exact).max()
    assert rel < 1e-9, rel
    st = ctx.stats()
    assert st["max_rel_residual"] <= 2e-12
    # true residual recomputed by the oracle
    op = OK.make_operator(m, gs.veff, gs.phi, shifts)
    assert OK.true_residual(op, X, B).max() <= 2e-12
    # iteration counts agree with the oracle's plain batched solver
    fn = OK.cg if solver == 0 else OK.minres
    _, it_ref, _ = fn(op, B, 1e-12)
    assert np.abs(iters.astype(int) - it_ref).max() <= 3
    ctx.close()


def test_sternheimer_default_tolerance_and_edge_cases():
    m, gs, B, shifts, exact = _rhs_batch(1)
    ctx = make_ctx(1, tol=1e-8)
    # a single system, and a zero right-hand side inside the batch
    X, it, _ = ctx.sternheimer(shifts[:1], to_dev(B[:, :1]))
    assert OK.true_residual(OK.make_operator(m, gs.veff, gs.phi, shifts[:1]), to_host(X), B[:, :1]).max() <= 1e-8
    B2 = B[:, :20].copy()
    B2[:, 3] = 0.0
    X2, it2, _ = ctx.sternheimer(shifts[:20], to_dev(B2))
    X2 = to_host(X2)
    assert it2[3] == 0 and np.all(X2[:, 3] == 0.0)
    res = OK.true_residual(OK.make_operator(m, gs.veff, gs.phi, shifts[:20]), X2, B2)
    res[3] = 0.0
    assert res.max() <= 1e-8
    ctx.close()
