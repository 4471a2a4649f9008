"""More than 256 orbitals: the Krylov vectors as column-major blocks and the
projector of Eq. (3.6) as two GEMMs (multi-shift CG, and CG per system),
against the oracle on a 48 x 48 grid with N_e = 300 and N_e = 1024
l2-orthonormal random orbitals.  The occupied energies are placed below the
spectrum of H, so every shifted operator Q (H - s) Q is positive definite on
range(Q); the oracle solves the compressed equations from the eigenpairs of
the projected operator and runs Alg. 2, Alg. 3, Alg. 4 and Sec. 2.2 step by step
with its own selections, which are forced on the GPU."""
import functools

import numpy as np
import pytest

from tests.gpu_common import grid_dict, require_gpu, to_dev, to_host
from oracle import acp as OA
from oracle import chi0 as OC
from oracle.model import build_model
from workload.seeds import draw_sketch, small_config

pytestmark = pytest.mark.gpu

CFG = small_config(903, 2, 4, 12, a=6.0, sigma=0.8, jitter=0.05, n_cheb=4, r=16)


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@functools.lru_cache(maxsize=None)
def _system(n_e):
    m = build_model(CFG)
    V = m.superposed_atoms_potential()
    H = m.hamiltonian_dense(V)
    lam_min = float(np.linalg.eigvalsh(H)[0])
    rng = np.random.default_rng(n_e)
    phi, _ = np.linalg.qr(rng.standard_normal((m.grid.n_grid, n_e)))
    eps = np.linspace(lam_min - 1.0, lam_min - 0.25, n_e)
    G = m.perturbations()
    om = draw_sketch(CFG, G.shape[1])
    solver = OA.ProjectedSpectralSolver(H, phi)
    return m, V, H, phi, eps, G, om, solver


def _ctx(n_e, **opts):
    from paper_1605_08021_amd import acp
    m, V, H, phi, eps, G, om, solver = _system(n_e)
    o = dict(n_cheb=CFG.n_cheb, n_mu=128, sketch_r=CFG.r, tol=1e-12, max_iter=5000)
    o.update(opts)
    print(f"[gpu] N_g={m.grid.n_grid} N_e={n_e} opts={o}", flush=True)
    return acp.Context(grid_dict(CFG), o, to_dev(phi), eps, to_dev(V))


@pytest.mark.parametrize("n_e", [300, 1024])
@pytest.mark.parametrize("solver_id", [0, 2])
def test_many_orbitals_dyson_dynmat_match_oracle(n_e, solver_id):
    m, V, H, phi, eps, G, om, solver = _system(n_e)
    kmax = 2
    ref = OA.acp_dyson(phi, eps, G, om, CFG.n_cheb, 128, solver, vc=m.vc, vc_inv=m.vc_inv, f=m.f,
                       dv=m.grid.dv, k_max=kmax)
    ctx = _ctx(n_e, solver=solver_id, dyson_max_iter=kmax)
    U, iters, _ = ctx.dyson(to_dev(G), to_dev(om), sel_hist_in=np.stack(ref.sel_hist))
    assert iters == kmax
    st = ctx.stats()
    last = ref.last
    ez = _rel(to_host(ctx.compress_get("z")), np.concatenate(last.Z, axis=1))
    ew = _rel(to_host(ctx.compress_get("w")), last.W)
    eu = float(np.linalg.norm(to_host(U) - ref.U) / np.linalg.norm(ref.U))
    K = np.random.default_rng(5).standard_normal((G.shape[1], G.shape[1]))
    K = K + K.T
    masses = np.ones(m.n_atoms)
    D, lam = ctx.dynmat(to_dev(G), None, K, masses)
    Dref, lamref = OC.dynamical_matrix(m.grid.dv * (G.T @ ref.U) + K, masses, CFG.dim)
    ed = float(np.linalg.norm(D - Dref) / np.linalg.norm(Dref))
    el = float(np.abs(lam - lamref).max() / np.abs(lamref).max())
    print(f"[wide] N_e={n_e} solver={solver_id}: Z {ez:.2e} W {ew:.2e} U {eu:.2e} D {ed:.2e} "
          f"omega^2 {el:.2e}; true residual {st['max_rel_residual']:.1e}, iterations "
          f"{st['iters_min']}-{st['iters_max']}", flush=True)
    ctx.close()
    assert st["max_rel_residual"] <= 2e-12
    assert ez <= 1e-9 and ew <= 1e-9 and eu <= 1e-9
    assert ed <= 1e-9 and el <= 1e-9


@pytest.mark.parametrize("n_e", [300, 1024])
def test_many_orbitals_sternheimer_per_column_shifts(n_e):
    """acp_sternheimer with a different shift in every column (one CG sequence
    each), including a zero right-hand side, against the dense oracle solve."""
    m, V, H, phi, eps, G, om, solver = _system(n_e)
    rng = np.random.default_rng(9)
    B = OA.project_q(phi, rng.standard_normal((m.grid.n_grid, 37)))
    B[:, 5] = 0.0
    sh = rng.uniform(eps[0], eps[-1], 37)
    ctx = _ctx(n_e)
    X, it, _ = ctx.sternheimer(sh, to_dev(B))
    X = to_host(X)
    Xref = np.stack([solver(float(sh[j]), B[:, j:j + 1])[:, 0] for j in range(37)], axis=1)
    err = float(np.abs(X - Xref).max() / np.abs(Xref).max())
    print(f"[wide] sternheimer N_e={n_e}: rel err {err:.2e}, iterations {it.min()}-{it.max()}", flush=True)
    assert it[5] == 0 and np.all(X[:, 5] == 0.0)
    assert err <= 1e-10
    assert ctx.stats()["max_rel_residual"] <= 2e-12
    ctx.close()


def test_many_orbitals_learned_fallback():
    """The learned form above 256 orbitals with a network that returns 0: every
    column breaks down at once and is finished by the FP64 per-system CG of the
    many-orbital form from its recomputed residual."""
    m, V, H, phi, eps, G, om, solver = _system(300)
    rng = np.random.default_rng(12)
    B = OA.project_q(phi, rng.standard_normal((m.grid.n_grid, 20)))
    sh = rng.uniform(eps[0], eps[-1], 20)
    ctx = _ctx(300, tol=1e-10)
    ctx.precond_init(3)
    ctx.precond_set(np.zeros(ctx.precond_n_params(), dtype=np.float32))
    ctx.set_opts(use_learned_precond=1)
    X, it, _ = ctx.sternheimer(sh, to_dev(B))
    X = to_host(X)
    Xref = np.stack([solver(float(sh[j]), B[:, j:j + 1])[:, 0] for j in range(20)], axis=1)
    err = float(np.abs(X - Xref).max() / np.abs(Xref).max())
    print(f"[wide] learned fallback: rel err {err:.2e}, iterations {it.min()}-{it.max()}, "
          f"fallback passes {ctx.stats()['refinements']}", flush=True)
    assert ctx.stats()["refinements"] >= 1
    assert err <= 1e-8
    ctx.close()
