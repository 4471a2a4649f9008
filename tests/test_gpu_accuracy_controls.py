"""Accuracy controls of the approximation (Sec. 3, Table 1 and Table 2 of the
paper, in trend): on the GPU, the error of U = chi G from ACP against the exact
response (the oracle's sum-over-states chi0 and dense Dyson) falls as the rank
N_mu grows at a fixed number of Chebyshev shifts, and as N_c grows at a fixed
rank; the phonon frequencies follow.  The paper's own values are for its
planewave model and are not reproduced by value."""
import functools

import numpy as np
import pytest

from tests.gpu_common import make_ctx, require_gpu, system, to_dev, to_host
from oracle import chi0 as OC
from oracle.model import yukawa_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@functools.lru_cache(maxsize=None)
def _exact(cid):
    cfg, m, gs, w, v, G, om, K = system(cid)
    X0 = OC.chi0_sos_matrix(m, w, v, gs.n_e)
    Vc = yukawa_dense(m.grid, m.kappa, m.eps0)
    U = OC.dyson_dense(X0, Vc, G)
    _, lam = OC.dynamical_matrix(OC.hessian_exact(m, gs, U, G), np.ones(m.n_atoms), cfg.dim)
    return U, lam


def _acp_error(cid, n_cheb, n_mu):
    cfg, m, gs, w, v, G, om, K = system(cid)
    Uex, lamex = _exact(cid)
    ctx = make_ctx(cid, n_cheb=n_cheb, n_mu=n_mu, tol=1e-12, dyson_max_iter=4)
    U, _, _ = ctx.dyson(to_dev(G), to_dev(om))
    _, lam = ctx.dynmat(to_dev(G), None, K, np.ones(m.n_atoms))
    ctx.close()
    eu = np.linalg.norm(to_host(U) - Uex) / np.linalg.norm(Uex)
    el = np.abs(lam - lamex).max() / np.abs(lamex).max()
    return eu, el


@pytest.mark.parametrize("cid", [11, 12])
def test_error_falls_with_rank_and_shifts(cid):
    ranks = [8, 16, 32, 64]
    by_rank = [_acp_error(cid, 8, r) for r in ranks]
    shifts = [2, 4, 8]
    by_shift = [_acp_error(cid, c, 64) for c in shifts]
    print(f"[acc] cfg {cid}: U / omega^2 error vs N_mu (N_c = 8): "
          + ", ".join(f"{r}: {e[0]:.1e}/{e[1]:.1e}" for r, e in zip(ranks, by_rank)), flush=True)
    print(f"[acc] cfg {cid}: U / omega^2 error vs N_c (N_mu = 64): "
          + ", ".join(f"{c}: {e[0]:.1e}/{e[1]:.1e}" for c, e in zip(shifts, by_shift)), flush=True)
    eu_r = [e[0] for e in by_rank]
    eu_c = [e[0] for e in by_shift]
    # the rank trend until the Chebyshev floor, the shift trend at full rank
    assert eu_r[0] > eu_r[1] > eu_r[2]
    assert eu_c[0] > eu_c[1] > eu_c[2]
    assert eu_c[-1] < 1e-2
