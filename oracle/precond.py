"""The learned preconditioner's network in plain FP64 (test infrastructure:
part of the oracle; the paper has no such network, so every definition here is
the specification the library's BF16 kernels are checked against).

Network N_theta: four circular (periodic) convolutions with kernels of width 5
along every grid axis (5 taps in 1D, 5 x 5 in 2D), channels 2 -> 32 -> 32 ->
32 -> 1, a bias per output channel, ReLU after the first three.  Inputs for a
residual r at shift s: channel 0 = r / rms(r), channel 1 = the constant
s_hat = (s - (eps_1 + eps_Ne)/2) / ((eps_Ne - eps_1)/2 + 1e-12).  The
correction it proposes is d = Q (N_theta(r) * rms(r)).

A convolution is a cross-correlation over the periodic grid:
    out[co, a] = b[co] + sum_ci sum_t W[co, ci, t] in[ci, a + off(t)],
1D: off(t) = t - 2;  2D (grid index a = ix + nx iy): t = 5 (dy + 2) + (dx + 2).

Parameter vector theta (also the weight format of the C ABI): for each layer in
order, W as [cout][cin][taps] then b as [cout].

Training (Adam on theta) minimises the mean over samples of the error of the
proposed correction in the energy norm of A (the norm CG minimises),
    (d - e)^T A (d - e) / e^T A e,   e = x* - x_k,  d = Q (N_theta(r) rms(r)),
for iterates x_k with residuals r_k = b - A x_k.  Since A e = r, it is written
    (d^T A d - 2 d^T r + e^T r) / e^T r,
which needs A only on d.  (The plain l2 error ||N_theta(r) - e/rms(r)||^2 /
||e/rms(r)||^2 is kept as `loss`/`loss_grad`; corrections trained on it keep
high-frequency errors that A amplifies, so they make poor preconditioners.)

Every function is the definition written out: the convolution as a sum of
rolled copies, the backward pass by the chain rule layer by layer.
"""
from __future__ import annotations

import numpy as np

CHANNELS = [(2, 32), (32, 32), (32, 32), (32, 1)]
WIDTH = 5


def n_taps(dim: int) -> int:
    return WIDTH if dim == 1 else WIDTH * WIDTH


def offsets(dim: int):
    """(dy, dx) of every tap, in tap order."""
    if dim == 1:
        return [(0, t - 2) for t in range(WIDTH)]
    return [(dy, dx) for dy in range(-2, 3) for dx in range(-2, 3)]


def n_params(dim: int) -> int:
    t = n_taps(dim)
    return sum(co * ci * t + co for ci, co in CHANNELS)


def unpack(theta, dim: int):
    """List of (W[cout, cin, taps], b[cout]) views into theta."""
    t = n_taps(dim)
    out, k = [], 0
    for ci, co in CHANNELS:
        W = theta[k:k + co * ci * t].reshape(co, ci, t)
        k += co * ci * t
        b = theta[k:k + co]
        k += co
        out.append((W, b))
    assert k == len(theta)
    return out


def init_params(dim: int, rng) -> np.ndarray:
    """He-style initial weights (uniform, fan-in scaled), zero biases."""
    t = n_taps(dim)
    parts = []
    for ci, co in CHANNELS:
        lim = np.sqrt(6.0 / (ci * t))
        parts.append(rng.uniform(-lim, lim, size=co * ci * t))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def shifted(x, shape, dy: int, dx: int):
    """x[..., a + off] on the periodic grid (x has the grid flattened last)."""
    lead = x.shape[:-1]
    g = x.reshape(lead + tuple(shape))
    if len(shape) == 1:
        g = np.roll(g, -dx, axis=-1)
    else:
        g = np.roll(np.roll(g, -dy, axis=-2), -dx, axis=-1)
    return g.reshape(lead + (-1,))


def conv(x, W, b, shape):
    """x [B, cin, N] -> [B, cout, N]."""
    dim = len(shape)
    out = np.zeros((x.shape[0], W.shape[0], x.shape[2]))
    for t, (dy, dx) in enumerate(offsets(dim)):
        xs = shifted(x, shape, dy, dx)                       # [B, cin, N]
        out += np.einsum("oi,bin->bon", W[:, :, t], xs)
    return out + b[None, :, None]


def conv_backward(x, W, gout, shape):
    """Gradients of conv w.r.t. its input, weights and bias, given dL/dout."""
    dim = len(shape)
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, (dy, dx) in enumerate(offsets(dim)):
        xs = shifted(x, shape, dy, dx)
        gW[:, :, t] = np.einsum("bon,bin->oi", gout, xs)
        # out[a] uses x[a + off]: the input gradient gathers gout[a - off]
        gx += shifted(np.einsum("oi,bon->bin", W[:, :, t], gout), shape, -dy, -dx)
    gb = gout.sum(axis=(0, 2))
    return gx, gW, gb


def features(R, shat):
    """Network input for residuals R [N, B] at normalised shifts shat [B]:
    [B, 2, N] and the rms of every column."""
    R = np.asarray(R, dtype=np.float64)
    rms = np.sqrt(np.mean(R * R, axis=0))
    safe = np.where(rms > 0, rms, 1.0)
    X = np.empty((R.shape[1], 2, R.shape[0]))
    X[:, 0, :] = (R / safe).T
    X[:, 1, :] = np.asarray(shat, dtype=np.float64)[:, None]
    return X, rms


def forward(theta, X, shape, dim: int):
    """Network output [B, 1, N] and the activations the backward pass needs."""
    layers = unpack(theta, dim)
    acts = [X]
    h = X
    for i, (W, b) in enumerate(layers):
        h = conv(h, W, b, shape)
        if i < len(layers) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def backward(theta, acts, gout, shape, dim: int):
    """dL/dtheta (same layout as theta) for dL/d(output) = gout [B, 1, N]."""
    layers = unpack(theta, dim)
    grads = [None] * len(layers)
    g = gout
    for i in range(len(layers) - 1, -1, -1):
        W, b = layers[i]
        if i < len(layers) - 1:
            g = g * (acts[i + 1] > 0.0)        # ReLU: acts[i+1] is its output
        gx, gW, gb = conv_backward(acts[i], W, g, shape)
        grads[i] = (gW, gb)
        g = gx
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def loss(out, T):
    """Mean over samples of ||out_b - T_b||^2 / ||T_b||^2 (out, T: [B, 1, N])."""
    d = out - T
    num = np.sum(d * d, axis=(1, 2))
    den = np.sum(T * T, axis=(1, 2))
    return float(np.mean(num / den))


def loss_grad(out, T):
    d = out - T
    den = np.sum(T * T, axis=(1, 2))
    return 2.0 * d / (den[:, None, None] * out.shape[0])


def energy_loss(out, rms, R, E, phi, apply_a):
    """Energy-norm loss of the corrections d = Q (out rms) for pairs (R, E)
    (columns; A E = R), and its gradient w.r.t. out ([B, 1, N]).
    apply_a applies A column by column."""
    B = out.shape[0]
    D = out[:, 0, :].T * rms[None, :]
    D = D - phi @ (phi.T @ D)
    AD = apply_a(D)
    er = np.sum(E * R, axis=0)
    per = (np.sum(D * AD, axis=0) - 2.0 * np.sum(D * R, axis=0) + er) / er
    G = 2.0 * (AD - R) / (er[None, :] * B)          # dL/dD (A symmetric)
    G = G - phi @ (phi.T @ G)                       # through Q
    return float(np.mean(per)), (G * rms[None, :]).T[:, None, :]


def targets(E, rms):
    """Training targets e / rms(r) as [B, 1, N]."""
    safe = np.where(rms > 0, rms, 1.0)
    return (np.asarray(E, dtype=np.float64) / safe).T[:, None, :]


def adam(theta, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def apply(theta, R, shat, phi, shape, dim: int):
    """Proposed corrections d = Q (N_theta(r) rms(r)) for residual columns R."""
    X, rms = features(R, shat)
    out, _ = forward(theta, X, shape, dim)
    D = out[:, 0, :].T * rms[None, :]
    return D - phi @ (phi.T @ D)


def shift_hat(shifts, eps_occ):
    lo, hi = float(eps_occ[0]), float(eps_occ[-1])
    return (np.asarray(shifts, dtype=np.float64) - 0.5 * (lo + hi)) / (0.5 * (hi - lo) + 1e-12)
