"""Dense symmetric eigensolver (cyclic Jacobi over the device) against the
library routine numpy.linalg.eigh: eigenvalues, eigenvector residuals and
orthonormality, on matrices with odd order (a bye in every round), repeated
and exactly zero eigenvalues (the acoustic modes of a dynamical matrix)."""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(-1.0, 3.0, n)
    lam[:3] = 0.0                      # a threefold zero eigenvalue
    lam[3:5] = 1.25                    # a degenerate pair
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), np.sort(lam)


@pytest.mark.parametrize("n", [7, 129, 300, 601])
def test_syev_matches_library(n):
    from paper_1605_08021_amd import acp
    A, lam = _matrix(n, n)
    print(f"[eig] n = {n}", flush=True)
    w, V = acp.syev(to_dev(A))
    ref = np.linalg.eigvalsh(A)
    scale = np.abs(ref).max()
    assert np.abs(w - ref).max() <= 1e-13 * n * scale
    V = to_host(V)
    assert np.abs(A @ V - V * w).max() <= 1e-12 * n * scale
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-13 * n
    w2, _ = acp.syev(to_dev(A), want_vectors=False)
    assert np.array_equal(w2, w)


@pytest.mark.parametrize("n", [600, 1025, 1500, 4096, 4097])
def test_gesv_matches_library(n):
    """Dense solve of the Dyson step: blocked LU (32-column panels up to 1024
    rows, 8-column panels of up to 4096 rows before them) and Gauss-Jordan
    above 4096, against numpy.linalg.solve on a nonsymmetric,
    well-conditioned matrix with a pivoting pattern (small diagonal)."""
    from paper_1605_08021_amd import acp
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + np.eye(n) * 0.01
    A = A + 2.0 * np.roll(np.eye(n), 1, axis=1)   # dominant superdiagonal: row exchanges
    B = rng.standard_normal((n, 7))
    print(f"[gesv] n = {n}", flush=True)
    X = to_host(acp.gesv(to_dev(A), to_dev(B)))
    ref = np.linalg.solve(A, B)
    cond = np.linalg.cond(A)
    err = np.abs(X - ref).max() / np.abs(ref).max()
    print(f"[gesv] n = {n}: cond {cond:.1e}, rel err {err:.1e}", flush=True)
    assert err <= 1e-15 * cond * n


@pytest.mark.parametrize("n_p", [129, 600, 2048])
def test_dynmat_eigenvalues_above_128(n_p):
    """acp_dynmat above 128 modes: Householder tridiagonalisation over the
    device and Sturm bisection, against the library routine on the D it returns
    (random G, U and local terms on workload 1's grid; 2048 is workload 5's
    count)."""
    from tests.gpu_common import make_ctx, to_dev
    rng = np.random.default_rng(n_p)
    ctx = make_ctx(1)
    ng = ctx.grid.n[0]
    G = rng.standard_normal((ng, n_p))
    U = rng.standard_normal((ng, n_p)) * 1e-2
    K = rng.standard_normal((n_p, n_p))
    K = K + K.T
    D, w2 = ctx.dynmat(to_dev(G), to_dev(U), K, None)
    ctx.close()
    ref = np.linalg.eigvalsh(0.5 * (D + D.T))
    err = float(np.abs(np.sort(w2) - ref).max() / np.abs(ref).max())
    print(f"[eig] dynmat n_p={n_p}: eigenvalue error {err:.1e}", flush=True)
    assert np.all(np.diff(w2) >= 0)
    assert err <= 1e-12
