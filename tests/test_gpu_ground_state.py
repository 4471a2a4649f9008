"""Lowest eigenpairs of H = -1/2 Delta_h + diag(V) on the GPU (Chebyshev-
filtered subspace iteration) against the oracle's eigensolvers (dense eigh on
small grids, shift-invert Lanczos on the sparse H above that) for the same
potential: eigenvalues, residuals under the oracle's own H, orthonormality and
the occupied subspace itself (its projector)."""
import numpy as np
import pytest

from tests.gpu_common import grid_dict, require_gpu, to_dev, to_host
from oracle.model import build_model
from workload.seeds import get_config, small_config

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


CASES = {
    "1d": (get_config(1), False),
    "2d_small": (small_config(901, 2, 3, 10, a=6.0, sigma=0.8, jitter=0.05), False),
    "2d_large": (small_config(902, 2, 9, 12, a=6.0, sigma=0.8, jitter=0.05), True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_lowest_eigenpairs_match_oracle(case):
    from paper_1605_08021_amd import acp
    cfg, sparse = CASES[case]
    m = build_model(cfg)
    V = m.superposed_atoms_potential()
    ref = m.ground_state_of(V, n_extra=1, sparse=sparse)
    n_e = m.n_e
    print(f"[gs] {case}: N_g={m.grid.n_grid} N_e={n_e}", flush=True)
    psi, lam, nxt, passes, res = acp.lowest_eigenpairs(grid_dict(cfg), to_dev(V), n_e, tol=1e-10, seed=5)
    Phi = to_host(psi)
    print(f"[gs] {case}: {passes} passes, largest residual {res:.2e}, "
          f"eigenvalue error {np.abs(lam - ref.eps[:n_e]).max():.2e}, next Ritz value {nxt:.6f} "
          f"(eigenvalue {ref.eps[n_e]:.6f})", flush=True)
    assert res <= 1e-10
    scale = max(1.0, np.abs(ref.eps[:n_e]).max())
    assert np.abs(lam - ref.eps[:n_e]).max() <= 1e-11 * scale
    HPhi = m.hamiltonian_apply(V, Phi)
    assert np.sqrt(((HPhi - Phi * lam) ** 2).sum(axis=0)).max() <= 2e-10
    assert np.abs(Phi.T @ Phi - np.eye(n_e)).max() <= 1e-12
    # same occupied subspace: the singular values of Phi_ref^T Phi are all 1
    sv = np.linalg.svd(ref.phi.T @ Phi, compute_uv=False)
    assert 1.0 - sv.min() <= 1e-10
    assert abs(nxt - ref.eps[n_e]) <= 1e-2 * max(1.0, abs(ref.eps[n_e]))


SCF_CASES = {
    "1d_paper": get_config(11),
    "2d_small": small_config(901, 2, 3, 10, a=6.0, sigma=0.8, jitter=0.05),
}


@pytest.mark.parametrize("case", list(SCF_CASES))
def test_scf_matches_oracle_fixed_point(case):
    """acp_scf reaches the oracle's self-consistent fixed point: density,
    effective potential, energies and the occupied subspace, and its orbitals
    are eigenvectors of the oracle's H for the GPU's potential."""
    from paper_1605_08021_amd import acp
    cfg = SCF_CASES[case]
    m = build_model(cfg)
    ref = m.scf(tol=1e-13)
    n_e = m.n_e
    print(f"[scf] {case}: N_g={m.grid.n_grid} N_e={n_e}", flush=True)
    psi, eps, veff, rho, it, res = acp.scf(grid_dict(cfg), to_dev(m.m), n_e, tol=1e-12, eig_tol=1e-11)
    Phi, V, rh = to_host(psi), to_host(veff), to_host(rho)
    sv = np.linalg.svd(ref.phi.T @ Phi, compute_uv=False)
    print(f"[scf] {case}: {it} iterations, residual {res:.1e}; rho {np.abs(rh - ref.rho).max():.1e}, "
          f"V {np.abs(V - ref.veff).max():.1e}, eps {np.abs(eps[:n_e] - ref.eps[:n_e]).max():.1e}, "
          f"subspace {1 - sv.min():.1e}", flush=True)
    assert res <= 1e-12
    assert np.abs(rh - ref.rho).max() <= 1e-9 * np.abs(ref.rho).max()
    assert np.abs(V - ref.veff).max() <= 1e-9 * max(1.0, np.abs(ref.veff).max())
    assert np.abs(eps[:n_e] - ref.eps[:n_e]).max() <= 1e-9
    assert 1.0 - sv.min() <= 1e-9
    H = m.hamiltonian_dense(V)
    assert np.abs(H @ Phi - Phi * eps[:n_e]).max() <= 1e-10


@pytest.mark.parametrize("case", [0, 1])
def test_scf_reproduces_paper_ground_state(case):
    """The paper's 60-atom 1D insulator and semiconductor (Sec. 4.1): the GPU
    SCF gives the printed gap and density range to the printed 4 digits."""
    import json
    import os
    from oracle.model import Grid, Model
    from paper_1605_08021_amd import acp
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_1d_ground_state.json")))
    c = gold["cases"][case]
    n_atoms, a, h = gold["model"]["n_atoms"], gold["model"]["a"], 0.1
    n = int(round(n_atoms * a / h))
    g = Grid((n,), n_atoms * a / n)
    R = ((np.arange(n_atoms) + 0.5) * a).reshape(-1, 1)
    m = Model(g, R, np.ones(n_atoms), n_atoms, sigma=0.3, kappa=0.1, eps0=c["eps0"], f=1.0)
    grid = dict(dim=1, n=(n,), h=g.h, kappa=0.1, eps0=c["eps0"], occ=1.0)
    psi, eps, veff, rho, it, res = acp.scf(grid, to_dev(m.m), n_atoms, tol=1e-10)
    rh = to_host(rho)
    gap = eps[n_atoms] - eps[n_atoms - 1]
    print(f"[scf] paper case {case}: {it} iterations; gap {gap:.5f} (printed {c['gap']}), "
          f"rho [{rh.min():.5f}, {rh.max():.5f}] (printed [{c['rho_min']}, {c['rho_max']}])", flush=True)
    half_ulp = 0.5 * 10.0 ** -c["printed_digits"]
    assert abs(gap - c["gap"]) <= half_ulp
    assert abs(rh.min() - c["rho_min"]) <= half_ulp
    assert abs(rh.max() - c["rho_max"]) <= half_ulp
