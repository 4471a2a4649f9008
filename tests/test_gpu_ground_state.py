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
