"""Benchmark: Sternheimer right-hand-side x shift systems solved per second.

One step = one pass of the whole ACP hot path on the workload: Alg. 4 with
k_max compressions (each: ISDF point selection, right-hand sides, the N_c N_mu
projected shifted solves to a relative residual of 1e-8, W), the Dyson updates,
then the dynamical matrix and its eigenvalues.  value = shifted systems solved
per second over the timed steps (whole job; inputs already in HBM).

Default workload: the 2D lattice of 32 x 32 sites on a 384 x 384 grid (1024
occupied orbitals, 2048 perturbations, N_c = 8, N_mu = 4096: 32768 shifted
systems per compression), one Dyson iteration per step (k_max = 1, so that the
driver's 25 steps fit its time limit; --dyson-iters sets more).

Input preparation (ground state by the library's GPU eigensolver, perturbations,
local Hessian terms) is done once, untimed, by paper_1605_08021_amd.workload_model.

Default form (more than 256 orbitals): the projector GEMMs in BF16 with FP32
accumulation on the deflated operator, FP64 vectors, every solution projected
and its residual recomputed in FP64; one step of the batched FP64 multi-shift
form is timed beside it and the difference of the two dynamical matrices
reported (--no-fp64-compare skips it).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--form auto|fast|bf16|mixed|learned|single|plain|batch|compress|dfpt]
                       [--no-cpu-baseline] [--no-fp64-compare] [--calibrate-copy]

--form batch: the uneven batch instead (16 ragged 1D chains and 16 ragged 2D
lattices with 5% vacancies; the shifted solves of each half share one
persistent launch, replayed from a hipGraph); one step = one compression of
every system; the same systems compressed one at a time are timed beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector and matrix), vendor figure
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 matrix, vendor figure


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


CSRC = os.path.join(ROOT, "paper_1605_08021_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mscg_kernel_cfg2_traffic.json")
KERNEL_SOURCES = [os.path.join(CSRC, f) for f in ("k_mscg.hip", "krylov_common.h")]
GEMM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_projector_cfg5_traffic.json")
GEMM_SOURCES = [os.path.join(CSRC, "k_gemm.hip")]
BF16_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_bf16_projector_cfg5_traffic.json")
BF16_SOURCES = [os.path.join(CSRC, "k_gemm_bf16.hip")]


def kernel_source_hash(sources=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, path: str = TRAFFIC_FILE, sources=None):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by the copy-kernel calibration), or None
    when the kernel source has changed since the counters were taken."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash(sources) or rec.get("workload") != workload:
        return None
    return rec.get("traffic_bytes_per_launch")


def calibrate_copy():
    """A plain device copy of known size, profiled beside the solver to scale the
    FETCH_SIZE / WRITE_SIZE counters: 3 copies of 256 MiB."""
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each": 8 * n, "copies": 3}), flush=True)


def cpu_baseline(inp, sample_cols: int, tol: float):
    """The oracle's plain batched CG (test infrastructure), timed on the host on a
    bounded sample of the same shifted systems.  Returns the JSON object."""
    import numpy as np
    from oracle import acp as OA
    from oracle import krylov as OK
    from oracle.model import Grid, Model

    cfg = inp.cfg
    grid = Grid(tuple(cfg.n), cfg.h)
    m = Model(grid, inp.R, inp.Z, inp.n_e, sigma=cfg.sigma, kappa=cfg.kappa, eps0=cfg.eps0,
              f=cfg.f)
    t0 = time.perf_counter()
    nodes, _ = OA.shifts_and_weights(inp.eps[: inp.n_e], cfg.n_cheb)
    per = max(1, sample_cols // len(nodes))
    if grid.n_grid * cfg.r * inp.n_e * 8 <= 4e9:
        # the first sample_cols // N_c right-hand sides of the oracle's own ISDF, every shift
        dec = OA.isdf_qrcp(inp.phi, inp.G, inp.omega, cfg.n_mu)
        R = OA.rhs(inp.phi, dec.xi)[:, :per]
        what = "right-hand sides of the oracle's ISDF"
    else:
        # the sketched M~ would not fit: right-hand sides -Q e_alpha at evenly
        # spaced grid points (interpolation vectors of the identity selection)
        E = np.zeros((grid.n_grid, per))
        E[np.linspace(0, grid.n_grid - 1, per).astype(int), np.arange(per)] = 1.0
        R = OA.rhs(inp.phi, E)
        what = "right-hand sides -Q e_alpha at evenly spaced grid points"
    t_prep = time.perf_counter() - t0
    B = np.tile(R, (1, len(nodes)))
    shifts = np.repeat(nodes, per)
    H = m.hamiltonian_sparse(inp.veff) if grid.n_grid > 20000 else None
    op = OK.make_operator(m, inp.veff, inp.phi, shifts, H=H)
    t0 = time.perf_counter()
    x, it, _ = OK.cg(op, B, tol)
    t = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": B.shape[1] / t, "unit": "systems/s", "cores": cores, "kind": "oracle",
            "sample": f"{B.shape[1]} of the {len(nodes) * cfg.n_mu} shifted systems of one "
                      f"compression ({per} {what} x {len(nodes)} shifts), plain batched "
                      f"CG to {tol:g}, numpy/OpenBLAS; mean iterations {float(it.mean()):.0f}; "
                      f"solve {t:.1f} s (right-hand-side preparation {t_prep:.1f} s not counted)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--form", choices=["auto", "fast", "bf16", "mixed", "learned", "single", "plain", "batch",
                                       "compress", "dfpt"],
                    default="auto", help="auto: bf16 above 256 orbitals, else fast")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="bf16 form: skip the FP64-form step timed beside it")
    ap.add_argument("--batch-systems", type=int, default=16, help="systems per dimension (--form batch)")
    ap.add_argument("--batch-dims", default="1,2", help="--form batch: 1, 2 or 1,2 (the 1D and 2D halves)")
    ap.add_argument("--dyson-iters", type=int, default=0, help="k_max (0: 1 for workload 5, else 4)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="CPU baseline systems (0: 256, 16 above 100k points)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the copy kernel used to calibrate the traffic counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the shifted systems are independent, see the design notes for sharding)",
              file=sys.stderr)
        sys.exit(2)
    if args.form == "batch":
        run_batch(args)
        return

    import numpy as np
    import torch
    from paper_1605_08021_amd import acp
    from paper_1605_08021_amd.workload_model import build_inputs
    from workload.seeds import get_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = get_config(args.config)
    if args.dyson_iters <= 0:
        args.dyson_iters = 1 if args.config == 5 else 4
    log(f"building inputs for workload {args.config}: {cfg.name}")
    t0 = time.perf_counter()
    inp = build_inputs(cfg)
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s; gap {inp.gap:.5f}, "
        f"self-consistent {inp.self_consistent}")
    dev = torch.device("cuda:0")
    if args.form == "auto":
        args.form = "bf16" if inp.n_e > 256 else "fast"

    def T(a):
        a = np.asarray(a, dtype=np.float64)
        if a.ndim == 2:
            return torch.from_numpy(np.ascontiguousarray(a.T)).to(dev).t()
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    phi, veff, G, om = T(inp.phi), T(inp.veff), T(inp.G), T(inp.omega)
    solver = {"fast": acp.SOLVER_CG, "bf16": acp.SOLVER_CG, "mixed": acp.SOLVER_CG,
              "single": acp.SOLVER_CG_SINGLE,
              "plain": acp.SOLVER_MINRES, "learned": acp.SOLVER_CG_SINGLE,
              "compress": acp.SOLVER_CG, "dfpt": acp.SOLVER_CG_SINGLE}[args.form]
    dfpt = args.form == "dfpt"
    compress_only = args.form == "compress"
    learned = args.form == "learned"
    mixed = args.form == "mixed"
    bf16 = args.form == "bf16"
    opts = dict(n_cheb=cfg.n_cheb, n_mu=cfg.n_mu, sketch_r=cfg.r, tol=args.tol, max_iter=20000,
                solver=solver, dyson_max_iter=args.dyson_iters,
                precision=(acp.PREC_FP32_REFINE if mixed else acp.PREC_BF16_PROJ if bf16 else acp.PREC_FP64),
                inner_tol=1e-5)
    ctx = acp.Context(dict(dim=cfg.dim, n=cfg.n, h=cfg.h, kappa=cfg.kappa, eps0=cfg.eps0,
                           occ=cfg.f), opts, phi, inp.eps[: inp.n_e], veff)
    masses = np.ones(inp.R.shape[0])
    train_info = None
    if learned:
        # untimed: the network is trained once, on the method's own solves for 16
        # right-hand sides at every shift of the first compression
        from paper_1605_08021_amd import precond as PC
        t0 = time.perf_counter()
        ctx.compress(G, om)
        Rfull = ctx.compress_get("rhs")
        shifts = ctx.shifts()
        cols = torch.arange(16, device=dev)
        B = torch.cat([Rfull[:, cols]] * len(shifts), dim=1)
        sh = np.repeat(shifts, 16)
        hist = PC.train_preconditioner(ctx, sh, B, seed=1234)
        ctx.set_opts(use_learned_precond=1)
        train_info = {"pairs_systems": int(B.shape[1]), "steps": int(sum(len(h) for h in hist)),
                      "loss_first": round(float(hist[0][:20].mean()), 4),
                      "loss_last": round(float(hist[-1][-20:].mean()), 4),
                      "seconds": round(time.perf_counter() - t0, 1)}
        log(f"preconditioner trained: {train_info}")

    def step():
        if compress_only:
            ctx.compress(G, om)
            return 1, None, None
        if dfpt:   # the comparator: Alg. 1 + Anderson-mixed Dyson to the same tolerance
            U, iters, _ = ctx.dfpt(G, max_iter=200, tol=args.tol, history=8, beta=0.5)
            D, w2 = ctx.dynmat(G, U, inp.K_local, masses)
            return iters, w2, D
        U, iters, _ = ctx.dyson(G, om)
        D, w2 = ctx.dynmat(G, U, inp.K_local, masses)
        return iters, w2, D

    for i in range(args.warmup):
        log(f"warmup step {i + 1}/{args.warmup}")
        step()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        iters, w2, D = step()
        log(f"step {i + 1}/{args.steps} done ({iters} compressions)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ctx.stats()
    fp64_form = None
    if bf16 and not args.no_fp64_compare:
        # the fastest FP64 form (batched FP64 multi-shift CG) on the same inputs:
        # one untimed and one timed step, and the difference of its dynamical matrix
        # and frequencies from the BF16 form's last step
        ctx.set_opts(precision=acp.PREC_FP64)
        log("FP64 form beside it: one untimed step")
        step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, w2_64, D64 = step()
        torch.cuda.synchronize()
        ms64 = 1e3 * (time.perf_counter() - t1)
        log(f"FP64 form step: {ms64:.1f} ms")
        fp64_form = {"form": "batched FP64 multi-shift CG, same workload and tolerance",
                     "ms_per_step": round(ms64, 2),
                     "speedup_of_bf16_form": round(ms64 / (1e3 * elapsed / args.steps), 3),
                     "rel_diff_D": float(np.linalg.norm(D - D64) / np.linalg.norm(D64)),
                     "max_rel_diff_omega2": float(np.abs(w2 - w2_64).max() / np.abs(w2_64).max())}
    systems = st["systems_solved"]
    value = systems / elapsed
    ms_step = 1e3 * elapsed / args.steps

    # roofline of the dominant kernel: the fused batched Krylov solver.  The library
    # accumulates the algorithmic bytes (vector sweeps x 8 B x N_g per system-iteration)
    # and the projector flops of every launch, and times each launch with HIP events
    # on its own stream.
    ng = inp.phi.shape[0]
    ne = inp.n_e
    launches = max(st["solve_kernel_launches"], 1)
    if st["ms_solve_kernel"] <= 0.0:
        st["ms_solve_kernel"] = float("nan")
    bytes_per_launch = st["krylov_bytes"] / launches
    flops_per_launch = st["krylov_flops"] / launches
    ms_per_launch = st["ms_solve_kernel"] / launches
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    kname = {acp.SOLVER_CG: "mscg_kernel (multi-shift CG: fused stencil + projector, shifted updates)"
             + (" FP32 storage, with per-system FP32 cg_kernel corrections" if mixed else ""),
             acp.SOLVER_MINRES: "minres_kernel (fused stencil + projector + MINRES)",
             acp.SOLVER_CG_SINGLE: "cg_kernel (fused stencil + projector + CG)"}[solver]
    traffic = (measured_traffic(f"config {args.config}")
               if solver == acp.SOLVER_CG and not mixed else None)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname,
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "mfma_fp64_tflops": round(flops_per_launch / (ms_per_launch * 1e-3) / 1e12, 2),
                "ms_per_launch": round(ms_per_launch, 3),
                "workgroups_per_tile": st["krylov_group"]}
    wide = ne > 256
    if wide:
        # many orbitals: the dominant kernel is the projector GEMM pair on the FP64
        # matrix cores (gemm_f64_kernel<.., 2>: C = Phi^T y, then y - Phi C), timed
        # by HIP events on the context's stream around the two launches of every
        # iteration; achieved = 4 N_g N_e flops per live column and iteration
        gemm_launches = 2 * launches
        tflops = st["krylov_flops"] / (st["ms_solve_kernel"] * 1e-3) / 1e12
        if bf16:
            # the same pair in BF16 (gemm_bf16_tn_kernel<2,2,0>: Phi^T p with both
            # operands in two terms, <3,1,0>: Phi (T - Lambda) C with Phi in three,
            # stored in FP32 for the stencil to add), timed together with the small
            # kernel between them; achieved = the same algorithmic 4 N_g N_e flops per
            # column and iteration, against the dense BF16 peak (the split terms
            # execute 3x as many)
            roofline = {"bound": "mfma", "achieved": round(tflops, 2), "peak": BF16_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tflops / BF16_PEAK_TFLOPS, 4),
                        "traffic": measured_traffic(f"config {args.config}", BF16_TRAFFIC_FILE, BF16_SOURCES),
                        "kernel": "gemm_bf16_tn_kernel<2,2,0> + <3,1,0> (projector GEMMs of the many-orbital "
                                  "multi-shift CG, v_mfma_f32_16x16x32_bf16, FP32 accumulation)",
                        "algorithmic_flops_per_launch": st["krylov_flops"] / gemm_launches,
                        "executed_mfma_tflops": round(3.0 * tflops, 2),
                        "algorithmic_bytes_per_launch": st["krylov_bytes"] / gemm_launches,
                        "ms_per_launch": round(st["ms_solve_kernel"] / gemm_launches, 3),
                        "iterations": launches}
    if wide and not bf16:
        roofline = {"bound": "mfma", "achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
                    "traffic": measured_traffic(f"config {args.config}", GEMM_TRAFFIC_FILE,
                                                GEMM_SOURCES),
                    "kernel": "gemm_f64_kernel<.., 2> (projector GEMMs of the many-orbital multi-shift CG, "
                              "FP64 v_mfma_f64_16x16x4)",
                    "algorithmic_flops_per_launch": st["krylov_flops"] / gemm_launches,
                    "algorithmic_bytes_per_launch": st["krylov_bytes"] / gemm_launches,
                    "ms_per_launch": round(st["ms_solve_kernel"] / gemm_launches, 3),
                    "iterations": launches}
    if learned:
        roofline = None   # no single fused kernel: the flexible CG is a host-driven loop
    log(f"stats: {json.dumps(st)}")
    out = {
        "metric": "Sternheimer RHS*shifts solved/s at 1e-8 residual",
        "value": round(value, 1),
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "bf16+f64" if bf16 else "f64",
        "data": "synthetic",
        "config": {"workload": f"config {args.config}: {cfg.name}; Harris (non-self-consistent) "
                               f"ground state{' from the GPU eigensolver' if ng > 8000 else ''}, "
                               f"gap {inp.gap:.5f} Ha",
                   "form": ("DFPT (Alg. 1 Sternheimer solves at the occupied energies, FP64 CG per system; "
                            "Dyson equation by Anderson mixing to the same tolerance) + dynamical matrix"
                            if dfpt else
                            "one compression per step (point selection, right-hand sides, "
                            "batched FP64 multi-shift CG, W); no Dyson update or dynamical matrix"
                            if compress_only else
                            "flexible CG with the learned BF16 conv preconditioner (FP64 vectors)"
                            if learned else
                            "batched multi-shift CG with the projector GEMMs in BF16 (FP32 accumulation) on the "
                            "deflated operator, FP64 stencil and vectors; every solution projected and its "
                            "residual recomputed in FP64"
                            if bf16 else
                            "FP32-storage multi-shift CG + FP64 iterative refinement") if (mixed or learned or compress_only or dfpt or bf16) else
                           {acp.SOLVER_CG: "batched FP64 multi-shift CG",
                            acp.SOLVER_CG_SINGLE: "batched FP64 CG, one sequence per system",
                            acp.SOLVER_MINRES: "plain FP64 MINRES"}[solver],
                   "dyson_iterations": st["dyson_iters"], "n_g": ng, "n_e": ne,
                   "n_p": int(inp.G.shape[1]), "n_c": cfg.n_cheb, "n_mu": cfg.n_mu,
                   "tol": args.tol},
        "max_true_rel_residual": st["max_rel_residual"],
        "refinements": st["refinements"],
        "preconditioner_training": train_info,
        "iters_min_max_last_solve": [st["iters_min"], st["iters_max"]],
        "phase_ms_per_step": {k: round(st[k] / args.steps, 2) for k in
                              ("ms_isdf", "ms_rhs", "ms_solve", "ms_residual", "ms_w",
                               "ms_dyson_small", "ms_dynmat")},
        "roofline": roofline,
    }
    if wide:
        # the Krylov vector kernels of the many-orbital solver (stencil, p.w, residual,
        # base update, deferred shifted updates): algorithmic bytes over their time
        # (each iteration's events minus the projector pair)
        if st["ms_vectors"] > 0:
            gbs = st["vector_bytes"] / (st["ms_vectors"] * 1e-3) / 1e9
            out["roofline_vector_kernels"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                              "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                              "bytes_per_step": st["vector_bytes"] / args.steps,
                                              "ms_per_step": round(st["ms_vectors"] / args.steps, 2)}
        out["fp64_form"] = fp64_form
    ctx.close()
    # release every device object before the interpreter's teardown (a profiler
    # preloaded into the process has finalised by then)
    del phi, veff, G, om
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle CG on a bounded sample)")
        sample = args.cpu_sample or (16 if inp.phi.shape[0] > 100000 else 256)
        out["cpu_baseline"] = cpu_baseline(inp, sample, args.tol)
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Uneven batch: every system's compression (point selection, right-hand sides,
    all shifted solves, W), the solves of all systems of one dimension in one
    persistent launch replayed from a hipGraph (the 1D chains and the 2D
    lattices are two batches: the fused kernel is specialised by stencil form);
    then the same systems one at a time."""
    import numpy as np
    import torch
    from paper_1605_08021_amd import acp
    from paper_1605_08021_amd.workload_model import build_inputs
    from workload.seeds import ragged_batch_configs, ragged_batch_configs_2d

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    def T(a):
        a = np.asarray(a, dtype=np.float64)
        if a.ndim == 2:
            return torch.from_numpy(np.ascontiguousarray(a.T)).to(dev).t()
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    dims = [int(d) for d in args.batch_dims.split(",")]
    halves = []   # per dimension: contexts, G, omega, sizes, batch
    t0 = time.perf_counter()
    for dim in dims:
        cfgs = (ragged_batch_configs(count=args.batch_systems, lo=16, hi=128) if dim == 1 else
                ragged_batch_configs_2d(count=args.batch_systems, lo=4, hi=12))
        ctxs, Gs, oms, sizes = [], [], [], []
        for cfg in cfgs:
            inp = build_inputs(cfg)
            ctxs.append(acp.Context(dict(dim=cfg.dim, n=cfg.n, h=cfg.h, kappa=cfg.kappa, eps0=cfg.eps0,
                                         occ=cfg.f),
                                    dict(n_cheb=cfg.n_cheb, n_mu=cfg.n_mu, sketch_r=cfg.r, tol=args.tol,
                                         max_iter=20000, solver=acp.SOLVER_CG),
                                    T(inp.phi), inp.eps[: inp.n_e], T(inp.veff)))
            Gs.append(T(inp.G))
            oms.append(T(inp.omega))
            sizes.append((int(inp.phi.shape[0]), int(inp.n_e), cfg.n_mu))
        log(f"{dim}D half: {len(cfgs)} systems ready ({time.perf_counter() - t0:.1f} s): "
            f"(N_g, N_e, N_mu) = {sizes}")
        halves.append((dim, ctxs, Gs, oms, sizes, acp.Batch(ctxs, use_graph=True)))
    ctxs = [c for h in halves for c in h[1]]
    sizes = [z for h in halves for z in h[4]]

    def timed(fn, steps):
        for c in ctxs:
            c.reset_stats()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    def batched():
        for _, _, Gs, oms, _, batch in halves:
            batch.compress(Gs, oms)

    def one_by_one():
        for _, cs, Gs, oms, _, _ in halves:
            for c, g, o in zip(cs, Gs, oms):
                c.compress(g, o)

    for i in range(max(args.warmup, 1)):
        log(f"warmup {i + 1}: batched and one at a time")
        batched()
        one_by_one()
    t_seq = timed(one_by_one, args.steps)
    t_bat = timed(batched, args.steps)
    stats = [c.stats() for c in ctxs]
    infos = [h[5].info() for h in halves]
    systems = sum(st["systems_solved"] for st in stats) / args.steps
    res = max(st["max_rel_residual"] for st in stats)
    kbytes = sum(st["krylov_bytes"] for st in stats) / args.steps
    kflops = sum(st["krylov_flops"] for st in stats) / args.steps
    ms_launch = sum(info["ms_last"] for info in infos)   # one launch per half and step
    achieved = kbytes / (ms_launch * 1e-3) / 1e9
    log(f"batch info: {json.dumps(infos)}")
    desc = {1: f"{args.batch_systems} 1D chains of 16-128 sites (40 points per site)",
            2: f"{args.batch_systems} 2D lattices of 4x4-12x12 sites (12x12 points per site)"}
    out = {
        "metric": "Sternheimer RHS*shifts solved/s at 1e-8 residual",
        "value": round(systems / t_bat, 1),
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(1e3 * t_bat, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uneven batch: " + " + ".join(desc[d] for d in dims)
                               + ", 5% vacancies, N_c=8, N_mu=4 N_e",
                   "form": "the shifted solves of all systems of one dimension in one persistent multi-shift "
                           "launch (one batch per dimension), hipGraph replay",
                   "systems": [{"n_g": a, "n_e": b, "n_mu": c} for a, b, c in sizes],
                   "tol": args.tol},
        "max_true_rel_residual": res,
        "one_at_a_time": {"value": round(systems / t_seq, 1), "ms_per_step": round(1e3 * t_seq, 2)},
        "batch": [{"dim": h[0], **{k: info[k] for k in ("n_tiles", "grid", "order", "tuned", "graph_replays",
                                                        "ms_last")}}
                  for h, info in zip(halves, infos)],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "mscg_batch_kernel (persistent work queue over the systems' tiles)",
                     "algorithmic_bytes_per_launch": kbytes / len(halves),
                     "mfma_fp64_tflops": round(kflops / (ms_launch * 1e-3) / 1e12, 2),
                     "ms_per_launch": round(ms_launch / len(halves), 3)},
    }
    for h in halves:
        h[5].close()
    for c in ctxs:
        c.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
