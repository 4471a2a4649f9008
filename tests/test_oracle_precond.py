"""Pins of the learned preconditioner's FP64 reference network (oracle/precond.py)
against library routines and the mathematics: the circular convolution against
scipy's wrap-mode correlation, the hand-written backward pass against central
finite differences, Adam's first step against its closed form."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import precond as P


@pytest.mark.parametrize("dim", [1, 2])
def test_conv_is_wrap_mode_correlation(dim):
    rng = np.random.default_rng(1)
    shape = (13,) if dim == 1 else (7, 9)
    n = int(np.prod(shape))
    t = P.n_taps(dim)
    x = rng.standard_normal((2, 3, n))
    W = rng.standard_normal((4, 3, t))
    b = rng.standard_normal(4)
    out = P.conv(x, W, b, shape)
    for bi in range(2):
        for co in range(4):
            ref = np.full(shape, b[co])
            for ci in range(3):
                img = x[bi, ci].reshape(shape)
                if dim == 1:
                    ref += ndimage.correlate1d(img, W[co, ci], mode="wrap")
                else:
                    ref += ndimage.correlate(img, W[co, ci].reshape(5, 5), mode="wrap")
            assert np.allclose(out[bi, co], ref.ravel(), rtol=0, atol=1e-12)


def test_conv_delta_kernel_is_a_shift():
    shape = (11,)
    x = np.arange(22, dtype=float).reshape(1, 2, 11)
    W = np.zeros((2, 2, 5))
    W[0, 0, 4] = 1.0          # tap 4: offset +2
    W[1, 1, 0] = 1.0          # tap 0: offset -2
    out = P.conv(x, W, np.zeros(2), shape)
    assert np.array_equal(out[0, 0], np.roll(x[0, 0], -2))
    assert np.array_equal(out[0, 1], np.roll(x[0, 1], 2))


@pytest.mark.parametrize("dim", [1, 2])
def test_backward_matches_finite_differences(dim):
    rng = np.random.default_rng(2 + dim)
    shape = (12,) if dim == 1 else (6, 5)
    n = int(np.prod(shape))
    theta = P.init_params(dim, rng)
    theta += 0.05 * rng.standard_normal(theta.shape)   # non-zero biases
    R = rng.standard_normal((n, 3))
    E = rng.standard_normal((n, 3))
    shat = np.array([-0.7, 0.1, 0.9])
    X, rms = P.features(R, shat)
    T = P.targets(E, rms)

    def f(th):
        out, _ = P.forward(th, X, shape, dim)
        return P.loss(out, T)

    out, acts = P.forward(theta, X, shape, dim)
    g = P.backward(theta, acts, P.loss_grad(out, T), shape, dim)
    assert g.shape == theta.shape
    idx = rng.choice(theta.size, size=120, replace=False)
    # every bias, and weights of every layer
    off = 0
    for ci, co in P.CHANNELS:
        off += co * ci * P.n_taps(dim)
        idx = np.concatenate([idx, np.arange(off, off + co)])
        off += co
    h = 1e-5
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_loss_gradient_and_zero_at_target():
    rng = np.random.default_rng(5)
    T = rng.standard_normal((3, 1, 10))
    assert P.loss(T.copy(), T) == 0.0
    out = rng.standard_normal(T.shape)
    g = P.loss_grad(out, T)
    h = 1e-6
    for k in range(5):
        i = np.unravel_index(rng.integers(out.size), out.shape)
        op, om = out.copy(), out.copy()
        op[i] += h
        om[i] -= h
        assert abs((P.loss(op, T) - P.loss(om, T)) / (2 * h) - g[i]) < 1e-8


def test_adam_first_step_closed_form():
    """m_hat = g and v_hat = g^2 after one step: every parameter moves by
    lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    new, m, v = P.adam(th, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_features_and_projected_apply():
    rng = np.random.default_rng(7)
    n = 20
    phi, _ = np.linalg.qr(rng.standard_normal((n, 3)))
    R = rng.standard_normal((n, 4))
    X, rms = P.features(R, np.zeros(4))
    assert np.allclose(rms, np.linalg.norm(R, axis=0) / np.sqrt(n))
    assert np.allclose(np.mean(X[:, 0, :] ** 2, axis=1), 1.0)
    theta = P.init_params(1, rng)
    D = P.apply(theta, R, np.zeros(4), phi, (n,), 1)
    assert np.abs(phi.T @ D).max() < 1e-12
    # the network is positively homogeneous in r through the rms scaling
    D2 = P.apply(theta, 3.0 * R, np.zeros(4), phi, (n,), 1)
    assert np.allclose(D2, 3.0 * D, rtol=1e-12, atol=1e-14)


def test_parameter_count():
    assert P.n_params(1) == (2 * 32 * 5 + 32) + 2 * (32 * 32 * 5 + 32) + (32 * 5 + 1)
    assert P.n_params(2) == (2 * 32 * 25 + 32) + 2 * (32 * 32 * 25 + 32) + (32 * 25 + 1)


def test_energy_loss_definition_and_gradient():
    """With A E = R the loss equals the energy-norm error ratio written out
    directly; its gradient w.r.t. the network output matches finite differences."""
    rng = np.random.default_rng(9)
    n, B = 15, 3
    phi, _ = np.linalg.qr(rng.standard_normal((n, 2)))
    Q = np.eye(n) - phi @ phi.T
    M = rng.standard_normal((n, n))
    A = Q @ (M @ M.T + n * np.eye(n)) @ Q          # SPD on range(Q)
    E = Q @ rng.standard_normal((n, B))
    R = A @ E
    out = rng.standard_normal((B, 1, n))
    rms = np.array([0.5, 2.0, 1.3])
    L, g = P.energy_loss(out, rms, R, E, phi, lambda X: A @ X)
    D = Q @ (out[:, 0, :].T * rms)
    direct = np.mean([(D[:, b] - E[:, b]) @ A @ (D[:, b] - E[:, b]) / (E[:, b] @ A @ E[:, b])
                      for b in range(B)])
    assert abs(L - direct) < 1e-12 * max(1.0, direct)
    h = 1e-6
    for k in range(6):
        i = np.unravel_index(rng.integers(out.size), out.shape)
        op, om = out.copy(), out.copy()
        op[i] += h
        om[i] -= h
        fd = (P.energy_loss(op, rms, R, E, phi, lambda X: A @ X)[0]
              - P.energy_loss(om, rms, R, E, phi, lambda X: A @ X)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd))
    # the exact correction d = e has zero loss
    Lz, _ = P.energy_loss((np.linalg.pinv(np.diag(rms)) @ E.T)[:, None, :], rms, R, E, phi,
                          lambda X: A @ X)
    assert abs(Lz) < 1e-12


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments equal g and g^2 at
    every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so after t steps
    theta = theta_0 - t lr g / (|g| + eps) exactly (up to rounding); a wrong
    bias-correction power or moment update breaks it after the first step."""
    rng = np.random.default_rng(11)
    th0 = rng.standard_normal(6)
    g = rng.standard_normal(6)
    th, m, v = th0.copy(), np.zeros(6), np.zeros(6)
    lr = 3e-3
    for t in range(1, 41):
        th, m, v = P.adam(th, g, m, v, t, lr=lr)
        assert np.allclose(th, th0 - t * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_adam_minimises_a_quadratic():
    """Adam on f(theta) = |theta - c|^2 / 2 (gradient theta - c) reaches c."""
    c = np.array([0.3, -1.2, 2.0])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 4001):
        th, m, v = P.adam(th, th - c, m, v, t, lr=1e-2)
    assert np.abs(th - c).max() < 1e-3
