"""Training data and training loop of the learned preconditioner (loop control
only: every solve, residual, forward/backward pass and Adam step runs in the
library through the C ABI).

Pairs come from the method's own shifted solves: for systems Q(H - s)Q x = b,
the iterates x_k of the fused CG after k iterations give residuals
r_k = b - A x_k and errors e_k = x* - x_k, with x* solved to a tight tolerance.
A network trained only on those sees different residuals once it drives the
iteration itself (they carry its own error patterns), so training continues on
pairs harvested along the preconditioned iteration's own trajectories
(steepest descent with the current network, run by the library), a few
rounds.  Torch here only slices and concatenates device arrays.
"""
from __future__ import annotations

import numpy as np


def harvest_pairs(ctx, shifts, B, ks=(0, 4, 8, 16, 32, 64), tol_star=1e-11):
    """(R, E, shifts) for every column of B at every iteration count in ks."""
    import torch
    shifts = np.asarray(shifts, dtype=np.float64)
    saved = (ctx.opts.tol, ctx.opts.max_iter, ctx.opts.solver, ctx.opts.use_learned_precond)
    ctx.set_opts(tol=tol_star, max_iter=max(20000, saved[1]), solver=2, use_learned_precond=0)
    xstar, _, _ = ctx.sternheimer(shifts, B)
    Rs, Es, Ss = [], [], []
    for k in ks:
        if k == 0:
            xk = torch.zeros_like(xstar)
        else:
            ctx.set_opts(tol=1e-300, max_iter=int(k))
            xk, _, _ = ctx.sternheimer(shifts, B, allow_noconv=True)
        Rs.append(ctx.residual(shifts, B, xk))
        Es.append(xstar - xk)
        Ss.append(shifts)
    ctx.set_opts(tol=saved[0], max_iter=saved[1], solver=saved[2], use_learned_precond=saved[3])
    R = torch.cat(Rs, dim=1)
    E = torch.cat(Es, dim=1)
    return R, E, np.concatenate(Ss)


def train(ctx, R, E, shifts, steps=300, batch=64, lr=2e-3, seed=0, log_every=0):
    """Adam on random mini-batches of the pairs; returns the batch losses."""
    rng = np.random.default_rng(seed)
    n = R.shape[1]
    losses = []
    for it in range(steps):
        idx = rng.choice(n, size=min(batch, n), replace=False)
        ti = __import__("torch").as_tensor(idx, device=R.device)
        loss = ctx.precond_train_step(shifts[idx], R[:, ti], E[:, ti], lr)
        losses.append(loss)
        if log_every and (it + 1) % log_every == 0:
            print(f"[precond] step {it + 1}/{steps} loss {np.mean(losses[-log_every:]):.4f}", flush=True)
    return np.asarray(losses)


def harvest_trajectory(ctx, shifts, B, xstar, steps=6):
    """Pairs (r_k, x* - x_k) along preconditioned steepest descent with the
    current network (d = M(r), alpha = r.d / d.Ad, x += alpha d), computed by the
    library (acp_precond_trajectory) in batches of at most 1024 systems."""
    import torch
    shifts = np.asarray(shifts, dtype=np.float64)
    n = B.shape[1]
    Rs, Es = [[] for _ in range(steps)], [[] for _ in range(steps)]
    for j0 in range(0, n, 1024):
        j1 = min(n, j0 + 1024)
        R, E = ctx.precond_trajectory(shifts[j0:j1], B[:, j0:j1], xstar[:, j0:j1], steps)
        m = j1 - j0
        for k in range(steps):
            Rs[k].append(R[:, k * m:(k + 1) * m])
            Es[k].append(E[:, k * m:(k + 1) * m])
    R = torch.cat([t for k in range(steps) for t in Rs[k]], dim=1)
    E = torch.cat([t for k in range(steps) for t in Es[k]], dim=1)
    return R, E, np.concatenate([shifts] * steps)


def solve_star(ctx, shifts, B, tol_star=1e-11):
    saved = (ctx.opts.tol, ctx.opts.max_iter, ctx.opts.solver, ctx.opts.use_learned_precond)
    ctx.set_opts(tol=tol_star, max_iter=max(20000, saved[1]), solver=2, use_learned_precond=0)
    xstar, _, _ = ctx.sternheimer(np.asarray(shifts, dtype=np.float64), B)
    ctx.set_opts(tol=saved[0], max_iter=saved[1], solver=saved[2], use_learned_precond=saved[3])
    return xstar


def train_preconditioner(ctx, shifts, B, seed=1234, steps=400, rounds=2, round_steps=300,
                         batch=64, lr=2e-3, log_every=0):
    """The full recipe: CG-iterate pairs, then `rounds` of trajectory pairs.
    Returns the loss history of every stage."""
    import torch
    ctx.precond_init(seed)
    R, E, S = harvest_pairs(ctx, shifts, B)
    hist = [train(ctx, R, E, S, steps=steps, batch=batch, lr=lr, seed=seed, log_every=log_every)]
    xstar = solve_star(ctx, shifts, B)
    for k in range(rounds):
        R2, E2, S2 = harvest_trajectory(ctx, shifts, B, xstar)
        R, E, S = torch.cat([R, R2], dim=1), torch.cat([E, E2], dim=1), np.concatenate([S, S2])
        hist.append(train(ctx, R, E, S, steps=round_steps, batch=batch, lr=lr / 2, seed=seed + k + 1,
                          log_every=log_every))
    return hist
