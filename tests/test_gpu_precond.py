"""GPU parity of the learned preconditioner's BF16 network against the FP64
reference network (oracle/precond.py): forward pass, projected application and
parameter gradients, on 1D and 2D periodic grids with ragged tiles; then what a
network trained on the method's own solves gains in the preconditioned CG."""
import numpy as np
import pytest

from tests.gpu_common import make_ctx, require_gpu, system, to_dev, to_host
from oracle import precond as P

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _synthetic_ctx(dim):
    """A context on a small grid (ragged against the 128-point tiles): the
    network needs only the grid, the projector an orthonormal block."""
    from paper_1605_08021_amd import acp
    shape = (203,) if dim == 1 else (21, 19)
    n = int(np.prod(shape))
    rng = np.random.default_rng(11)
    phi, _ = np.linalg.qr(rng.standard_normal((n, 5)))
    eps = np.array([-0.9, -0.7, -0.6, -0.4, -0.3])
    grid = dict(dim=dim, n=list(shape[::-1]) if dim == 2 else [shape[0]], h=0.5, kappa=0.01,
                eps0=1.0, occ=2.0)
    ctx = acp.Context(grid, dict(n_cheb=4, n_mu=4, sketch_r=4), to_dev(phi), eps, to_dev(np.zeros(n)))
    return ctx, shape, phi, eps, rng


def _bf16(x):
    """Round to BF16 (nearest even), through FP32 as the kernels do."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _forward_bf16(theta, X, shape, dim):
    """The reference network with the kernels' storage rounding: BF16 weights
    and inputs, FP32 biases, BF16 hidden activations (after the ReLU)."""
    h = _bf16(X)
    layers = P.unpack(theta, dim)
    for i, (W, b) in enumerate(layers):
        h = P.conv(h, _bf16(W), b, shape)
        if i < len(layers) - 1:
            h = _bf16(np.maximum(h, 0.0))
    return h


def _grads_bf16(theta, X, rms, R, E, phi, apply_a, shape, dim):
    """Parameter gradients with the kernels' roundings: BF16 weights and stored
    activations, BF16 gradients between layers (ReLU mask from the stored
    activation), FP32-stored output."""
    layers = P.unpack(theta, dim)
    Wr = [_bf16(W) for W, _ in layers]
    acts = [_bf16(X)]
    h = acts[0]
    for i, (W, b) in enumerate(layers):
        h = P.conv(h, Wr[i], b, shape)
        if i < len(layers) - 1:
            h = _bf16(np.maximum(h, 0.0))
        acts.append(h)
    out = np.asarray(acts[-1], dtype=np.float32).astype(np.float64)
    _, gout = P.energy_loss(out, rms, R, E, phi, apply_a)
    g = _bf16(gout)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        gx, gW, gb = P.conv_backward(acts[i], Wr[i], g, shape)
        grads[i] = np.concatenate([gW.ravel(), gb])
        if i > 0:
            g = _bf16(gx * (acts[i] > 0.0))
    return np.concatenate(grads)


def _operator(shape, phi, shifts):
    """A_j = Q (-1/2 Delta_h - s_j) Q on the synthetic grid (V_eff = 0, h = 0.5)."""
    from oracle.model import Grid, laplacian_apply
    grid = Grid(tuple(shape[::-1]), 0.5)

    def apply(X):
        Xq = X - phi @ (phi.T @ X)
        Y = -0.5 * laplacian_apply(grid, Xq) - Xq * shifts[None, :]
        return Y - phi @ (phi.T @ Y)
    return apply


# Tolerances from the arithmetic: BF16 keeps 8 significant bits (unit roundoff
# u = 2^-8); each of the 4 layers rounds its weights and its input activations,
# relative error <= u/2 each, so the FP64 network is matched to 8 u/2 ~ 1.6e-2
# (2e-2); against the reference with the same roundings only the FP32
# accumulation order and the rare activation that rounds the other way remain.
TOL_FP64 = 2e-2
TOL_EMUL = 2e-3


def _theta(dim, rng):
    th = P.init_params(dim, rng)
    th += 0.02 * rng.standard_normal(th.shape)      # non-zero biases
    return th.astype(np.float32)


@pytest.mark.parametrize("dim", [1, 2])
def test_forward_and_apply_match_oracle(dim):
    ctx, shape, phi, eps, rng = _synthetic_ctx(dim)
    th = _theta(dim, rng)
    ctx.precond_set(th)
    assert np.array_equal(ctx.precond_get(), th)
    n = int(np.prod(shape))
    R = rng.standard_normal((n, 6))
    R[:, 3] *= 1e-7                                   # scale invariance
    shifts = np.array([-0.9, -0.3, -0.5, -0.6, -0.85, -0.4])
    shat = P.shift_hat(shifts, eps)
    X, rms = P.features(R, shat)
    ref, _ = P.forward(th.astype(np.float64), X, shape, dim)
    emul = _forward_bf16(th.astype(np.float64), X, shape, dim)
    out = to_host(ctx.precond_forward(shifts, to_dev(R)).double())
    for j in range(6):
        e, ee = _rel(out[j], ref[j, 0]), _rel(out[j], emul[j, 0])
        print(f"dim {dim} sample {j}: forward rel err {e:.2e} (vs BF16-rounded reference {ee:.2e})")
        assert e < TOL_FP64 and ee < TOL_EMUL
    D = to_host(ctx.precond_apply(shifts, to_dev(R)))
    Dref = P.apply(th.astype(np.float64), R, shat, phi, shape, dim)
    assert np.abs(phi.T @ D).max() <= 1e-12 * np.abs(D).max()
    assert _rel(D, Dref) < TOL_FP64
    ctx.close()


@pytest.mark.parametrize("dim", [1, 2])
def test_gradients_match_oracle(dim):
    """Energy-norm loss and parameter gradients of one training step (lr = 0)
    against the FP64 network and against the same network with the kernels'
    BF16 roundings; then one Adam step of size lr."""
    ctx, shape, phi, eps, rng = _synthetic_ctx(dim)
    th = _theta(dim, rng)
    ctx.precond_set(th)
    n = int(np.prod(shape))
    shifts = np.array([-0.9, -0.3, -0.5, -0.6, -0.85])
    A = _operator(shape, phi, shifts)
    E = rng.standard_normal((n, 5))
    E -= phi @ (phi.T @ E)
    R = A(E)
    shat = P.shift_hat(shifts, eps)
    loss, g = ctx.precond_train_step(shifts, to_dev(R), to_dev(E), 0.0, want_grad=True)
    X, rms = P.features(R, shat)
    out, acts = P.forward(th.astype(np.float64), X, shape, dim)
    lref, gout = P.energy_loss(out, rms, R, E, phi, A)
    gref = P.backward(th.astype(np.float64), acts, gout, shape, dim)
    gem = _grads_bf16(th.astype(np.float64), X, rms, R, E, phi, A, shape, dim)
    print(f"dim {dim}: loss {loss:.6f} (FP64 network {lref:.6f})")
    assert abs(loss - lref) <= TOL_FP64 * abs(lref)
    off = 0
    for l, (ci, co) in enumerate(P.CHANNELS):
        nw = co * ci * P.n_taps(dim)
        sl = slice(off, off + nw + co)
        e, ee = _rel(g[sl], gref[sl]), _rel(g[sl], gem[sl])
        print(f"dim {dim} layer {l}: grad rel err {e:.2e} (vs BF16-rounded reference {ee:.2e})")
        # the gradient passes through twice the roundings of the forward pass
        assert e < 3 * TOL_FP64 and ee < TOL_EMUL
        off += nw + co
    # lr = 0 leaves the parameters unchanged; one Adam step moves them by ~lr
    assert np.array_equal(ctx.precond_get(), th)
    ctx.precond_train_step(shifts, to_dev(R), to_dev(E), 1e-3)
    step = ctx.precond_get() - th
    assert np.abs(step).max() <= 1.01e-3 and np.abs(step).max() >= 0.9e-3
    ctx.close()


def test_training_and_what_the_network_gains():
    """Pairs (r_k, x* - x_k) from the fused CG's own iterates on workload 1
    (right-hand sides 0..15 at every shift), then from the preconditioned
    iteration's own trajectories, train the 1D network; on the other right-hand
    sides the preconditioned flexible CG reaches the same FP64 true residual as
    the same CG without the network in several times fewer iterations."""
    import torch
    from oracle import acp as OA, krylov as OK
    from paper_1605_08021_amd import precond as PC
    cfg, m, gs, w, v, G, om, K = system(1)
    dec = OA.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    nodes, _ = OA.shifts_and_weights(gs.eps[:gs.n_e], cfg.n_cheb)
    R0 = OA.rhs(gs.phi, dec.xi)
    train_cols, test_cols = np.arange(0, 16), np.arange(16, 32)
    Btr = np.concatenate([R0[:, train_cols]] * len(nodes), axis=1)
    str_ = np.repeat(nodes, len(train_cols))
    ctx = make_ctx(1, tol=1e-8, max_iter=5000)
    hist = PC.train_preconditioner(ctx, str_, to_dev(Btr), seed=1234)
    first, last = hist[0][:20].mean(), hist[-1][-20:].mean()
    print(f"training loss {first:.3f} -> {last:.3f} (energy norm)")
    assert last < 0.1 * first
    Bte = np.concatenate([R0[:, test_cols]] * len(nodes), axis=1)
    ste = np.repeat(nodes, len(test_cols))
    op = OK.make_operator(m, gs.veff, gs.phi, ste)
    res = {}
    for mode in (2, 1):
        ctx.set_opts(use_learned_precond=mode)
        X, it, _ = ctx.sternheimer(ste, to_dev(Bte))
        tr = OK.true_residual(op, to_host(X), Bte).max()
        res[mode] = (it.astype(float), tr)
        print(f"mode {mode}: iterations mean {it.mean():.1f} max {it.max()}, true residual {tr:.2e}")
        assert tr <= 1e-8
    gain = res[2][0].mean() / res[1][0].mean()
    print(f"iterations without / with the network: {gain:.2f}")
    assert gain > 2.0
    ctx.close()


@pytest.mark.parametrize("net", ["untrained", "zero"])
def test_bad_network_falls_back_to_fp64(net):
    """A network that was never trained (random weights) or one that returns 0:
    the flexible CG stalls or breaks down (p.Ap = 0) in those columns, which are
    then finished in FP64 MINRES from their recomputed residual, so the answer
    is the one of plain CG to the same tolerance."""
    from oracle import acp as OA, krylov as OK
    cfg, m, gs, w, v, G, om, K = system(1)
    dec = OA.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    nodes, _ = OA.shifts_and_weights(gs.eps[:gs.n_e], cfg.n_cheb)
    R0 = OA.rhs(gs.phi, dec.xi)
    cols = np.arange(0, 12)
    B = np.concatenate([R0[:, cols]] * len(nodes), axis=1)
    sh = np.repeat(nodes, len(cols))
    op = OK.make_operator(m, gs.veff, gs.phi, sh)
    ctx = make_ctx(1, tol=1e-8, max_iter=5000)
    ctx.precond_init(99)
    if net == "zero":
        ctx.precond_set(np.zeros(ctx.precond_n_params(), dtype=np.float32))
    ctx.set_opts(use_learned_precond=2)
    X2, it2, _ = ctx.sternheimer(sh, to_dev(B))
    ctx.set_opts(use_learned_precond=1)
    ctx.reset_stats()
    X1, it1, st = ctx.sternheimer(sh, to_dev(B))
    fell_back = ctx.stats()["refinements"]
    X1, X2 = to_host(X1), to_host(X2)
    tr = OK.true_residual(op, X1, B).max()
    diff = float(np.abs(X1 - X2).max() / np.abs(X2).max())
    print(f"[fallback] {net} network: iterations {it1.min()}-{it1.max()} (plain CG {it2.min()}-{it2.max()}), "
          f"fallback passes {fell_back}, true residual {tr:.2e}, vs plain CG {diff:.2e}", flush=True)
    assert tr <= 1e-8
    assert diff <= 1e-6
    if net == "zero":
        assert fell_back >= 1
    ctx.close()


def test_trajectory_matches_reference():
    """acp_precond_trajectory (steepest descent with the network, in the library)
    against the same three steps written here with the library's network and
    operator and the vector arithmetic in torch."""
    import torch
    from oracle import acp as OA
    cfg, m, gs, w, v, G, om, K = system(1)
    dec = OA.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    nodes, _ = OA.shifts_and_weights(gs.eps[:gs.n_e], cfg.n_cheb)
    B = np.concatenate([OA.rhs(gs.phi, dec.xi)[:, :6]] * 2, axis=1)
    sh = np.repeat(nodes[:2], 6)
    ctx = make_ctx(1, tol=1e-11, max_iter=5000)
    ctx.precond_init(7)
    Bd = to_dev(B)
    xstar, _, _ = ctx.sternheimer(sh, Bd)
    R, E = ctx.precond_trajectory(sh, Bd, xstar, 3)
    x = torch.zeros_like(Bd)
    r = Bd.clone()
    n = B.shape[1]
    for k in range(3):
        er = float((R[:, k * n:(k + 1) * n] - r).abs().max() / r.abs().max())
        ee = float((E[:, k * n:(k + 1) * n] - (xstar - x)).abs().max() / xstar.abs().max())
        print(f"[trajectory] step {k}: R {er:.2e} E {ee:.2e}", flush=True)
        assert er <= 1e-12 and ee <= 1e-12
        d = ctx.precond_apply(sh, r)
        Ad = ctx.residual(sh, torch.zeros_like(d), d).neg_()
        alpha = (r * d).sum(0) / (d * Ad).sum(0)
        x = x + alpha * d
        r = r - alpha * Ad
    ctx.close()


def _lattice_2d(cid, k):
    """A square lattice of k x k sites (spacing 6, sigma 0.8, 12 x 12 points per
    site, as workload 3) with its superposed-atom ground state."""
    from oracle import acp as OA
    from oracle.model import build_model
    from workload.seeds import small_config
    cfg = small_config(cid, 2, k, 12, a=6.0, sigma=0.8, jitter=0.05, n_cheb=8, r=16)
    m = build_model(cfg)
    V = m.superposed_atoms_potential()
    w, v = np.linalg.eigh(m.hamiltonian_dense(V))
    phi, eps = v[:, :m.n_e].copy(), w[:m.n_e].copy()
    G = m.perturbations()
    from workload.seeds import draw_sketch
    dec = OA.isdf_qrcp(phi, G, draw_sketch(cfg, G.shape[1]), 4 * m.n_e)
    return cfg, m, V, phi, eps, OA.rhs(phi, dec.xi)


def test_2d_network_transfers_to_a_larger_lattice():
    """a9 in 2D: the network trained on the solves of a 4 x 4 lattice (2304 grid
    points) is loaded into the context of a 6 x 6 lattice (5184 points) and
    preconditions its shifted systems: the same FP64 true residual as CG without
    the network in fewer iterations."""
    from paper_1605_08021_amd import acp
    from paper_1605_08021_amd import precond as PC
    from oracle import acp as OA, krylov as OK
    from tests.gpu_common import grid_dict
    out = []
    for cid, k in ((951, 4), (952, 6)):
        cfg, m, V, phi, eps, R0 = _lattice_2d(cid, k)
        ctx = acp.Context(grid_dict(cfg), dict(n_cheb=cfg.n_cheb, n_mu=4 * m.n_e, sketch_r=cfg.r, tol=1e-8,
                                               max_iter=5000), to_dev(phi), eps, to_dev(V))
        nodes, _ = OA.shifts_and_weights(eps, cfg.n_cheb)
        out.append((cfg, m, V, phi, eps, R0, ctx, nodes))
    (cfg_a, m_a, V_a, phi_a, eps_a, R_a, ctx_a, nodes_a), (cfg_b, m_b, V_b, phi_b, eps_b, R_b, ctx_b, nodes_b) = out
    cols = np.arange(16)
    Btr = np.concatenate([R_a[:, cols]] * len(nodes_a), axis=1)
    hist = PC.train_preconditioner(ctx_a, np.repeat(nodes_a, len(cols)), to_dev(Btr), seed=4321)
    print(f"[2d] trained on the 4x4 lattice: loss {hist[0][:20].mean():.3f} -> {hist[-1][-20:].mean():.3f}")
    ctx_b.precond_init(1)
    ctx_b.precond_set(ctx_a.precond_get())
    Bte = np.concatenate([R_b[:, cols]] * len(nodes_b), axis=1)
    ste = np.repeat(nodes_b, len(cols))
    op = OK.make_operator(m_b, V_b, phi_b, ste)
    res = {}
    for mode in (2, 1):
        ctx_b.set_opts(use_learned_precond=mode)
        ctx_b.reset_stats()
        X, it, _ = ctx_b.sternheimer(ste, to_dev(Bte))
        tr = OK.true_residual(op, to_host(X), Bte).max()
        res[mode] = (it.mean(), tr, ctx_b.stats()["refinements"])
        print(f"[2d] 6x6 lattice, mode {mode}: iterations mean {it.mean():.1f} max {it.max()}, "
              f"true residual {tr:.2e}, fallback passes {res[mode][2]}", flush=True)
        assert tr <= 1e-8
    gain = res[2][0] / res[1][0]
    print(f"[2d] iterations without / with the transferred network: {gain:.2f}")
    assert gain > 1.5
    ctx_a.close()
    ctx_b.close()


def test_flexible_cg_after_a_multishift_solve_on_one_context():
    """The host-driven CG's pinned open-column counters outlive a compression on
    the same context (whose fused multi-shift solve allocates its own pinned
    staging): the plain flexible CG run before and after it gives the same
    answer bit for bit, at the FP64 tolerance."""
    from oracle import acp as OA, krylov as OK
    cfg, m, gs, w, v, G, om, K = system(1)
    dec = OA.isdf_qrcp(gs.phi, G, om, cfg.n_mu)
    nodes, _ = OA.shifts_and_weights(gs.eps[:gs.n_e], cfg.n_cheb)
    R0 = OA.rhs(gs.phi, dec.xi)
    cols = np.arange(0, 12)
    B = np.concatenate([R0[:, cols]] * len(nodes), axis=1)
    sh = np.repeat(nodes, len(cols))
    op = OK.make_operator(m, gs.veff, gs.phi, sh)
    ctx = make_ctx(1, tol=1e-8, max_iter=5000)
    ctx.set_opts(use_learned_precond=2)
    Xa = to_host(ctx.sternheimer(sh, to_dev(B))[0])
    ctx.set_opts(use_learned_precond=0)
    ctx.compress(to_dev(G), to_dev(om))
    ctx.set_opts(use_learned_precond=2)
    Xb = to_host(ctx.sternheimer(sh, to_dev(B))[0])
    tr = OK.true_residual(op, Xb, B).max()
    print(f"[fcg after compress] true residual {tr:.2e}", flush=True)
    assert np.array_equal(Xa, Xb)
    assert tr <= 1e-8
    ctx.close()
