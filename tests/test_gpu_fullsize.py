"""The benchmark workload at its full size (N_g = 5120, N_e = 128, N_c = 8,
N_mu = 512: 4096 shifted systems), in the launch configuration the bench times
(autotuned group size and lockstep, suspensions with compaction planned from
the previous solve of the shape).  The oracle's operator Q (H - s) Q, built
from the oracle model on the same grid and the same seeded inputs, recomputes
the residual of sampled shifted solutions on the CPU; properties that hold at
any size are checked on all columns: the solutions lie in range(Q), and the
interpolation vectors are the identity at the selected points.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def test_workload2_sampled_residuals_and_properties():
    import torch
    from oracle import krylov as OK
    from oracle.model import build_model
    from paper_1605_08021_amd import acp
    from paper_1605_08021_amd.workload_model import build_inputs
    from workload.seeds import get_config

    cfg = get_config(2)
    inp = build_inputs(cfg)
    m = build_model(cfg)
    assert m.grid.n_grid == inp.phi.shape[0]
    dev = torch.device("cuda:0")

    def T(a):
        a = np.asarray(a, dtype=np.float64)
        if a.ndim == 2:
            return torch.from_numpy(np.ascontiguousarray(a.T)).to(dev).t()
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    print("[full] workload 2: compress (4096 shifted systems, tol 1e-8)", flush=True)
    ctx = acp.Context(dict(dim=cfg.dim, n=cfg.n, h=cfg.h, kappa=cfg.kappa, eps0=cfg.eps0, occ=cfg.f),
                      dict(n_cheb=cfg.n_cheb, n_mu=cfg.n_mu, sketch_r=cfg.r, tol=1e-8, max_iter=20000,
                           solver=acp.SOLVER_CG),
                      T(inp.phi), inp.eps[:inp.n_e], T(inp.veff))
    ctx.compress(T(inp.G), T(inp.omega))
    # the second solve of the shape plans its suspensions and compactions from
    # the iteration counts of the first, as every solve of the bench does
    ctx.reset_stats()
    print("[full] workload 2: second compress (planned suspensions)", flush=True)
    sel = np.asarray(ctx.compress(T(inp.G), T(inp.omega)))
    st = ctx.stats()
    print(f"[full] launches {st['solve_kernel_launches']}, last group size {st['krylov_group']}, "
          f"iterations {st['iters_min']}-{st['iters_max']}, "
          f"library true residual {st['max_rel_residual']:.3e}", flush=True)
    assert st["max_rel_residual"] <= 1e-8 * (1 + 1e-6)
    nmu, nc = cfg.n_mu, cfg.n_cheb
    R = to_host(ctx.compress_get("rhs"))     # -Q xi, N_g x N_mu
    Z = to_host(ctx.compress_get("z"))       # N_g x (N_c N_mu), block c = shift c
    Xi = to_host(ctx.compress_get("xi"))
    shifts = np.asarray(ctx.shifts())
    ctx.close()
    assert len(np.unique(sel)) == nmu
    assert np.array_equal(Xi[sel], np.eye(nmu))
    phi = np.asarray(inp.phi, dtype=np.float64)[:, :inp.n_e]
    # every solution lies in range(Q): the occupied component left by rounding
    # over ~300 iterations stays two orders below the solve tolerance
    occ = np.abs(phi.T @ Z).max(axis=0) / np.abs(Z).max(axis=0)
    print(f"[full] largest occupied component {occ.max():.2e}", flush=True)
    assert occ.max() < 1e-10, occ.max()
    # sampled systems: CPU residual of the oracle's operator
    for c in (0, nc // 2, nc - 1):
        for mu in (0, 137, 300, nmu - 1):
            z = Z[:, c * nmu + mu:c * nmu + mu + 1]
            b = R[:, mu:mu + 1]
            A = OK.make_operator(m, inp.veff, phi, [shifts[c]])
            res = float(OK.true_residual(A, z, b)[0])
            print(f"[full] shift {c} (eps~ = {shifts[c]:+.5f}), mu {mu}: CPU residual {res:.3e}", flush=True)
            assert res <= 1.05e-8
