"""Benchmark: seconds per all-at-once solve to a 1e-8 float64 relative residual,
mixed precision against float64 inner solves, with the shifted-stencil roofline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|medium]
                    [--p 20] [--no-cpu-baseline] [--mode solve|kernels|batch|exact|sp|blocks|paper|warmstart]

One step = one FGMRES(7) solve of calA x = b (b = (b_1, 0, ..., 0)) from x = 0
on resident device inputs, preconditioned by the nested-Chebyshev block
alpha-circulant preconditioner.  Prints ONE JSON line.

Workloads (synthetic, seeded):
* large  (default): 2048 x 2048 grid, kappa = 50 exp(g), g a Gaussian random
  field (std 1, correlation length 10 cells), l = 10, alpha = 1e-2, p = 20 inner
  steps per shift, complex64 inner with bfloat16 kappa, float64 outer.
* medium: the same on 512 x 512.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# sources that decide the three-step sweep's traffic: its device body and launch files, and
# the host code that picks its tiling
TRIPLE_SOURCES = ["stencil_triple.h", "stencil_kernels.h", "stencil_triple.hip", "tiling.h"]

WORKLOADS = {
    "large": {"nx": 2048, "ny": 2048, "ell": 10, "alpha": 1e-2, "kappa0": 50.0, "std": 1.0, "corr": 10.0},
    "medium": {"nx": 512, "ny": 512, "ell": 10, "alpha": 1e-2, "kappa0": 50.0, "std": 1.0, "corr": 10.0},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--p", type=int, default=20)
    ap.add_argument("--restart", type=int, default=None,
                    help="FGMRES restart length (default: 7 for the solve mode, 8 for the others)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-budgets", action="store_true", help="skip the p = 5 and p = 10 solves")
    ap.add_argument("--no-warm-start", action="store_true", help="skip training and timing the learned warm start")
    ap.add_argument("--no-const-check", action="store_true",
                    help="skip the constant-coefficient solves checked against the oracle's closed form")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--step-pairs", type=int, default=1, choices=[0, 1],
                    help="fuse two steady Chebyshev steps per sweep (1) or run single steps (0)")
    ap.add_argument("--pair-tiling", type=int, nargs=3, default=[0, 0, 0], metavar=("ROWS", "WPB", "VX"),
                    help="tiling of the paired sweep (0 = automatic)")
    ap.add_argument("--step-triples", type=int, default=1, choices=[0, 1],
                    help="fuse three steady Chebyshev steps per sweep (1) or at most two (0)")
    ap.add_argument("--triple-tiling", type=int, nargs=3, default=[0, 0, 0], metavar=("ROWS", "OCC", "VX"),
                    help="tiling of the three-step sweep (0 = automatic)")
    ap.add_argument("--mode", default="solve",
                    choices=["solve", "kernels", "batch", "exact", "sp", "blocks", "paper", "warmstart"],
                    help="kernels: only a few preconditioner applications plus a 512 MiB device copy "
                         "(the launch set used for hardware-counter runs); batch: many uneven problems "
                         "solved one by one and as one batch")
    ap.add_argument("--sp-iters", type=int, nargs="*", default=None,
                    help="sp mode: inner MINRES / CG iteration counts to time")
    ap.add_argument("--ws-nx", type=int, default=1024, help="warmstart mode: grid side")
    ap.add_argument("--ws-pairs", type=int, default=20000, help="warmstart mode: training crops")
    ap.add_argument("--ws-steps", type=int, default=4000, help="warmstart mode: Adam steps")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-restart", type=int, default=30,
                    help="FGMRES restart of the batch mode (p = 10: restart 8 leaves one of the 64 problems unconverged)")
    ap.add_argument("--tile-cache", default="", help="tiling cache file for the batch mode's tuner")
    a = ap.parse_args()
    if a.restart is None:
        # FGMRES(7) is the fastest restart for the default solve with fused Chebyshev
        # steps and for the warm-started one; the other modes were measured with FGMRES(8)
        a.restart = {"solve": 7, "warmstart": 7}.get(a.mode, 8)
    return a


def batch_mode(a):
    """Uneven batch: grid sides from {128, 256, 512, 1024}, l from {6, 8, 10, 12},
    kappa = 50 exp(g) with field std uniform in [0.5, 1.5] (correlation length 10),
    alpha = 1e-2, p = 10, FGMRES(30) to 1e-8, complex64 inner with bfloat16 kappa.
    Tiles come from the tuner; every problem is solved once alone (one after the
    other) and then all together with ac_batch_solve."""
    import tempfile

    import torch
    from paper_2506_03947_amd import api
    from synth import batched_problem_specs, first_block_rhs, lognormal_kappa
    L = api.L
    dev = torch.device("cuda:0")
    specs = batched_problem_specs(a.batch_count, seed=2026)
    ctx = api.ac_ctx_create(0)
    api.ac_ctx_set_step_pairs(ctx, a.step_pairs, *a.pair_tiling)
    api.ac_ctx_set_step_triples(ctx, a.step_triples, *a.triple_tiling)
    probs, bs = [], []
    for i, sp in enumerate(specs):
        kap = lognormal_kappa(sp["nx"], sp["ny"], 50.0, 10.0, sp["std"], seed=sp["seed"])
        probs.append(api.ac_problem_create(ctx, 2, sp["nx"], sp["ny"], torch.from_numpy(kap).to(dev), sp["ell"],
                                           1e-2))
        bs.append(torch.from_numpy(first_block_rhs(sp["nx"] * sp["ny"], sp["ell"], seed=i)).to(dev))
    log(f"{len(probs)} problems, {sum(p.ell * p.n for p in probs) / 1e6:.1f} M unknowns")
    prec = L.AC_PREC_MIXED_BF16K
    opts = api.Opts(precision=prec, p=10, tol=a.tol, restart_m=a.batch_restart, max_outer=3000)
    cache = a.tile_cache or os.path.join(tempfile.mkdtemp(), "tiles.json")
    pws = api.workspace(max(api.ac_prec_workspace_size(p, opts) for p in probs))
    t0 = time.perf_counter()
    tiles = [api.ac_tune_tiling(p, prec, pws, cache)[0] for p in probs]
    t_tune = time.perf_counter() - t0
    del pws
    xs = [torch.zeros(p.ell * p.n, dtype=torch.float64, device=dev) for p in probs]
    sws = api.workspace(max(api.ac_solve_workspace_size(p, opts) for p in probs))
    api.ac_solve(probs[0], opts, bs[0], xs[0], sws)  # warm-up
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single, t_each = [], []
    for p, b, x in zip(probs, bs, xs):
        t1 = time.perf_counter()
        single.append(api.ac_solve(p, opts, b, x, sws))
        t_each.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"one by one: {t_seq:.3f} s")
    # algorithmic bytes of the whole path (profiled repeat of the one-by-one solves)
    api.ac_ctx_set_profiling(ctx, True)
    api.ac_ctx_reset_stats(ctx)
    ys = [torch.zeros_like(x) for x in xs]
    for p, b, y in zip(probs, bs, ys):
        api.ac_solve(p, opts, b, y, sws)
    stats = api.ac_ctx_kernel_stats(ctx)
    api.ac_ctx_set_profiling(ctx, False)
    del ys, sws
    nbytes = sum(v["bytes"] for v in stats.values())
    bws = api.workspace(api.ac_batch_workspace_size(ctx, probs, opts))
    zs = [torch.zeros_like(x) for x in xs]
    times = []
    for rep in range(1 + max(a.steps, 1)):
        for z in zs:
            z.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = api.ac_batch_solve(ctx, probs, opts, bs, zs, bws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"batch run {rep}: {times[-1]:.3f} s")
    t_batch = min(times[1:])
    diff = max(float(torch.linalg.norm(z - x) / torch.linalg.norm(x)) for z, x in zip(zs, xs))
    its_b = [i["outer_iters"] for i in infos]
    its_s = [i["outer_iters"] for i in single]
    print(json.dumps({
        "metric": "batched all-at-once solves per second to 1e-8 (uneven grids and l)", "value": len(probs) / t_batch,
        "unit": "solves/s", "n_gpus": 1, "steps": len(times) - 1, "warmup": 1, "ms_per_step": 1000 * t_batch,
        "higher_is_better": True, "dtype": "c64/bf16 inner, f64 outer", "data": "synthetic",
        "config": {"workload": f"{len(probs)} problems, sides {{128,256,512,1024}}, l {{6,8,10,12}}, alpha 1e-2, "
                               f"p 10, FGMRES({a.batch_restart})", "unknowns": int(sum(p.ell * p.n for p in probs))},
        "one_by_one": {"value": len(probs) / t_seq, "seconds": t_seq},
        "speedup_vs_one_by_one": t_seq / t_batch,
        "aggregate": {"algorithmic_bytes": nbytes, "GBs": nbytes / t_batch / 1e9,
                      "frac_hbm": nbytes / t_batch / 1e9 / HBM_PEAK_GBS},
        "iterations": {"batch_max": max(its_b), "batch_sum": sum(its_b), "single_sum": sum(its_s),
                       "all_converged": all(i["converged"] for i in infos)},
        "max_rel_diff_batch_vs_single": diff, "tune_seconds": t_tune,
        "per_problem": [{"side": sp["nx"], "ell": sp["ell"], "iters": i["outer_iters"], "single_s": round(t, 5)}
                        for sp, i, t in zip(specs, single, t_each)],
        "tilings": sorted({tuple(t) for t in tiles}),
    }))


def exact_mode(a):
    """Constant coefficient kappa = 50 on the 2048 x 2048 grid, l = 10, alpha = 1e-2:
    FGMRES(restart) to 1e-8 with the exact P_alpha (inner float64 and float32) against
    the nested-Chebyshev P_NC (p inner steps, complex64 / bfloat16 kappa) on the same
    problem.  Reports seconds per solve, outer iterations and the per-application cost
    of the exact inner solve (forward and inverse sine transforms, each two half-size
    GEMMs of 2 (ceil(n_x/2)^2 + floor(n_x/2)^2) (n_y planes) flops, planes = real slots
    + 2 complex slots)."""
    import torch
    from paper_2506_03947_amd import api
    from synth import first_block_rhs
    L = api.L
    dev = torch.device("cuda:0")
    nx = ny = 2048
    ell, alpha, kappa = 10, 1e-2, 50.0
    n = nx * ny
    ctx = api.ac_ctx_create(0)
    prob = api.ac_problem_create(ctx, 2, nx, ny, torch.full((n,), kappa, dtype=torch.float64, device=dev), ell,
                                 alpha)
    b = torch.from_numpy(first_block_rhs(n, ell, seed=a.seed)).to(dev)
    planes = prob.ns + (prob.ns - (2 if ell % 2 == 0 else 1))  # real slots once, complex twice
    h, h2 = (nx + 1) // 2, nx // 2
    # forward and inverse sine transforms, each two half-size GEMMs (even / odd modes)
    gemm_flops = 2 * 2.0 * (h * h + h2 * h2) * ny * planes
    out = {}
    cases = {"exact_f64": api.Opts(precision=L.AC_PREC_FP64, inner=L.AC_INNER_EXACT, tol=a.tol,
                                   restart_m=a.restart, max_outer=3000),
             "exact_f32": api.Opts(precision=L.AC_PREC_MIXED_FP32K, inner=L.AC_INNER_EXACT, tol=a.tol,
                                   restart_m=a.restart, max_outer=3000),
             "nested_cheb_p%d" % a.p: api.Opts(precision=L.AC_PREC_MIXED_BF16K, p=a.p, tol=a.tol,
                                               restart_m=a.restart, max_outer=3000)}
    for name, opts in cases.items():
        ws = api.workspace(api.ac_solve_workspace_size(prob, opts))
        x = torch.zeros_like(b)
        api.ac_solve(prob, opts, b, x, ws)  # warm-up (library kernels load here)
        times = []
        for _ in range(max(a.steps, 1)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = api.ac_solve(prob, opts, b, x, ws)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        api.ac_ctx_set_profiling(ctx, True)
        api.ac_ctx_reset_stats(ctx)
        x.zero_()
        api.ac_solve(prob, opts, b, x, ws)
        st = api.ac_ctx_kernel_stats(ctx)
        api.ac_ctx_set_profiling(ctx, False)
        rec = {"seconds": min(times), "outer_iters": info["outer_iters"], "converged": info["converged"],
               "rel_residual": info["rel_residual_true"]}
        if opts.inner == L.AC_INNER_EXACT:
            e = st["exact"]
            per = e["ms"] / max(e["launches"], 1)
            rec.update({"exact_apply_ms": per, "gemm_flops_per_apply": gemm_flops,
                        "gemm_TFLOPs_lower_bound": gemm_flops / per / 1e9})
        log(f"{name}: {rec}")
        out[name] = rec
        del ws
    f64 = out["exact_f64"]
    print(json.dumps({
        "metric": "seconds per all-at-once solve to 1e-8, exact P_alpha (constant kappa)", "value": f64["seconds"],
        "unit": "s/solve", "n_gpus": 1, "steps": max(a.steps, 1), "warmup": 1, "ms_per_step": 1000 * f64["seconds"],
        "higher_is_better": False, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2048x2048 constant kappa 50, l 10, alpha 1e-2, FGMRES(%d)" % a.restart},
        "roofline": {"bound": "mfma", "achieved": f64["gemm_TFLOPs_lower_bound"], "peak": 78.6,
                     "unit": "TFLOP/s", "frac": f64["gemm_TFLOPs_lower_bound"] / 78.6, "traffic": None,
                     "note": "whole exact inner solve (GEMMs, tridiagonal, split/merge, inverse time-DFT) "
                             "timed against the GEMM flops only"},
        "cases": out,
    }), flush=True)


def sp_mode(a):
    """The default workload (2048 x 2048 log-normal kappa, l = 10, alpha = 1e-2,
    FGMRES(restart) to 1e-8) with the saddle-point preconditioner P_SP (Section 4:
    MINRES / CG inner solves, multigrid P_D; float64, and float32 vectors and multigrid
    coefficients) at a few inner iteration counts."""
    import torch
    from paper_2506_03947_amd import api
    from synth import first_block_rhs, lognormal_kappa
    L = api.L
    dev = torch.device("cuda:0")
    w = WORKLOADS[a.workload]
    nx, ny, ell, alpha = w["nx"], w["ny"], w["ell"], w["alpha"]
    n = nx * ny
    kap = lognormal_kappa(nx, ny, w["kappa0"], w["corr"], w["std"], seed=a.seed)
    ctx = api.ac_ctx_create(0)
    prob = api.ac_problem_create(ctx, 2, nx, ny, torch.from_numpy(kap).to(dev), ell, alpha)
    t0 = time.perf_counter()
    api.ac_problem_create_multigrid(prob)
    t_setup = time.perf_counter() - t0
    b = torch.from_numpy(first_block_rhs(n, ell, seed=a.seed)).to(dev)
    out = {}
    runs = [(prec, iters) for prec in (L.AC_PREC_FP64, L.AC_PREC_MIXED_FP32K) for iters in (a.sp_iters or [5, 8])]
    for prec, iters in runs:
        opts = api.Opts(precision=prec, inner=L.AC_INNER_SP, p=iters, tol=a.tol, restart_m=a.restart,
                        max_outer=3000)
        ws = api.workspace(api.ac_solve_workspace_size(prob, opts))
        x = torch.zeros_like(b)
        api.ac_solve(prob, opts, b, x, ws)
        times = []
        for _ in range(max(a.steps, 1)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = api.ac_solve(prob, opts, b, x, ws)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        api.ac_ctx_set_profiling(ctx, True)
        api.ac_ctx_reset_stats(ctx)
        x.zero_()
        api.ac_solve(prob, opts, b, x, ws)
        st = api.ac_ctx_kernel_stats(ctx)
        api.ac_ctx_set_profiling(ctx, False)
        sd = st["saddle"]
        rec = {"seconds": min(times), "outer_iters": info["outer_iters"], "converged": info["converged"],
               "rel_residual": info["rel_residual_true"], "matvecs_A": info["matvecs_A"],
               "prec_apply_ms": sd["ms"] / max(sd["launches"], 1)}
        key = ("f64_" if prec == L.AC_PREC_FP64 else "f32_") + str(iters)
        log(f"P_SP {key} inner iterations: {rec}")
        out[key] = rec
        del ws
    best = min(out.values(), key=lambda r: r["seconds"])
    print(json.dumps({
        "metric": "seconds per all-at-once solve to 1e-8, saddle-point preconditioner P_SP", "value": best["seconds"],
        "unit": "s/solve", "n_gpus": 1, "steps": max(a.steps, 1), "warmup": 1,
        "ms_per_step": 1000 * best["seconds"], "higher_is_better": False, "dtype": "f32 or f64 inner, f64 outer",
        "data": "synthetic",
        "config": {"workload": f"{nx}x{ny} log-normal kappa, l {ell}, alpha {alpha}, FGMRES({a.restart}), P_SP"},
        "multigrid_setup_s": t_setup, "inner_iterations": out,
    }), flush=True)


def blocks_mode(a):
    """Varying diagonal blocks A_1..A_l (the representative block A(mean kappa) in the
    preconditioner): the default grid, l = 10, alpha = 1e-2, kappa_k = 50 exp(g + d (k/l) h)
    for drifts d in {0, 0.5, 1}; FGMRES(restart) to 1e-8 with the nested-Chebyshev P
    (p inner steps, complex64 / bf16 kappa) and with P_SP (8 steps, float64).  Reports
    seconds and iterations per solve and the block-varying calA kernel's bandwidth."""
    import torch
    from paper_2506_03947_amd import api
    from synth import drifting_kappa_blocks, first_block_rhs
    L = api.L
    dev = torch.device("cuda:0")
    w = WORKLOADS[a.workload]
    nx, ny, ell, alpha = w["nx"], w["ny"], w["ell"], w["alpha"]
    n = nx * ny
    ctx = api.ac_ctx_create(0)
    b = torch.from_numpy(first_block_rhs(n, ell, seed=a.seed)).to(dev)
    out = {}
    for drift in (0.0, 0.5, 1.0):
        kb = drifting_kappa_blocks(nx, ny, ell, w["kappa0"], w["corr"], w["std"], drift, seed=a.seed)
        prob = api.ac_problem_create_blocks(ctx, 2, nx, ny, torch.from_numpy(kb.reshape(-1)).to(dev), ell, alpha)
        api.ac_problem_create_multigrid(prob)
        del kb
        # the nested-Chebyshev P(A_hat) stalls for strongly drifting blocks: cap its iterations
        cases = {"nested_cheb": api.Opts(precision=L.AC_PREC_MIXED_BF16K, p=a.p, tol=a.tol, restart_m=a.restart,
                                         max_outer=1000),
                 "saddle_sp8": api.Opts(precision=L.AC_PREC_FP64, inner=L.AC_INNER_SP, p=8, tol=a.tol,
                                        restart_m=a.restart, max_outer=3000)}
        for name, opts in cases.items():
            ws = api.workspace(api.ac_solve_workspace_size(prob, opts))
            x = torch.zeros_like(b)
            api.ac_ctx_set_profiling(ctx, True)
            api.ac_ctx_reset_stats(ctx)
            api.ac_solve(prob, opts, b, x, ws)  # warm-up, profiled
            st = api.ac_ctx_kernel_stats(ctx)["apply_calA"]
            api.ac_ctx_set_profiling(ctx, False)
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = api.ac_solve(prob, opts, b, x, ws)
            torch.cuda.synchronize()
            rec = {"seconds": time.perf_counter() - t0, "outer_iters": info["outer_iters"],
                   "converged": info["converged"], "rel_residual": info["rel_residual_true"],
                   "calA_GBps": st["bytes"] / st["ms"] / 1e6 if st["ms"] > 0 else None}
            log(f"drift {drift} {name}: {rec}")
            out[f"drift{drift}_{name}"] = rec
            del ws
        del prob
        torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "seconds per all-at-once solve to 1e-8, varying diagonal blocks (drift 0.5)", "value":
            out["drift0.5_nested_cheb"]["seconds"], "unit": "s/solve", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1000 * out["drift0.5_nested_cheb"]["seconds"], "higher_is_better": False,
        "dtype": "c64+bf16 (inner), f64 (outer)", "data": "synthetic",
        "config": {"workload": f"{nx}x{ny}, l {ell} drifting log-normal blocks, alpha {alpha}, FGMRES({a.restart})"},
        "cases": out,
    }), flush=True)


def paper_mode(a):
    """The paper's high-dimension comparison (Section 5): the paper operator
    A = I - (nu/h^2) L on n_x^2 grids, n_x in {500, 750, 1000, 1250, 1500}, l = 10,
    alpha = 0.01, b = (b_1, 0, ...), outer Chebyshev with the Corollary 1 interval to 1e-6;
    P_NC2 with the Algorithm 1 allocation of the budget l n_x eta, eta = 0.2 (float64 and
    complex64 with float32 kappa), and P_SP with 14 MINRES / CG steps per shift (the paper's matvec counts imply
    about 14).  Times, outer iterations and matvecs next to the paper's table."""
    import torch
    from paper_2506_03947_amd import api
    from synth import first_block_rhs
    L = api.L
    dev = torch.device("cuda:0")
    ell, alpha, eta, D = 10, 0.01, 0.2, 0.2
    paper = {500: (7, 7035, 2, 532), 750: (7, 10535, 2, 516), 1000: (7, 14056, 2, 516), 1250: (7, 17535, 2, 532),
             1500: (6, 18030, 2, 516)}
    ctx = api.ac_ctx_create(0)
    out = {}
    for nx in sorted(paper):
        n = nx * nx
        h = 1.0 / (nx + 1)
        kap = D * D / (2 * ell - 4) / (h * h)
        # exact constant-coefficient interval (Appendix A)
        lo = 1.0 + kap * 2.0 * 4.0 * np.sin(np.pi / (2 * (nx + 1))) ** 2
        hi = 1.0 + kap * 2.0 * 4.0 * np.cos(np.pi / (2 * (nx + 1))) ** 2
        prob = api.ac_problem_create(ctx, 2, nx, nx, torch.full((n,), kap, dtype=torch.float64, device=dev), ell,
                                     alpha, bounds=(lo, hi))
        api.ac_problem_create_multigrid(prob)
        b = torch.from_numpy(first_block_rhs(n, ell, seed=0)).to(dev)
        pm = api.ac_alloc_nc2(prob, ell * nx * eta)
        cases = {"nc2_f64": api.Opts(precision=L.AC_PREC_FP64, p=pm, tol=1e-6, restart_m=1, max_outer=200,
                                     outer=L.AC_OUTER_CHEBYSHEV),
                 # the outer Chebyshev iteration refuses bf16 kappa (its interval is too narrow)
                 "nc2_mixed": api.Opts(precision=L.AC_PREC_MIXED_FP32K, p=pm, tol=1e-6, restart_m=1, max_outer=200,
                                       outer=L.AC_OUTER_CHEBYSHEV),
                 "sp14": api.Opts(precision=L.AC_PREC_FP64, inner=L.AC_INNER_SP, p=14, tol=1e-6, restart_m=1,
                                  max_outer=200, outer=L.AC_OUTER_CHEBYSHEV)}
        row = {}
        for name, opts in cases.items():
            ws = api.workspace(api.ac_solve_workspace_size(prob, opts))
            x = torch.zeros_like(b)
            api.ac_solve(prob, opts, b, x, ws)
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = api.ac_solve(prob, opts, b, x, ws)
            torch.cuda.synchronize()
            row[name] = {"seconds": time.perf_counter() - t0, "outer_iters": info["outer_iters"],
                         "matvecs_A": info["matvecs_A"], "converged": info["converged"]}
            del ws
        row["paper"] = {"nc2_iters": paper[nx][0], "nc2_matvecs": paper[nx][1], "sp_iters": paper[nx][2],
                        "sp_matvecs": paper[nx][3]}
        log(f"n_x {nx}: {row}")
        out[str(nx)] = row
        del prob
        torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "seconds per outer-Chebyshev solve to 1e-6, paper operator, n_x = 1500 (P_SP)",
        "value": out["1500"]["sp14"]["seconds"], "unit": "s/solve", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1000 * out["1500"]["sp14"]["seconds"], "higher_is_better": False, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "paper operator, n_x 500..1500, l 10, alpha 0.01, eta 0.2"},
        "rows": out}), flush=True)


def train_warm_start(api, ctx, restart, p_in, n_target, steps, nx=1024, ell=10, alpha=1e-2):
    """Trains the warm-start network on the GPU with the library's kernels, on pairs the
    plain method generates: the first 60 vectors FGMRES(restart) hands to the
    preconditioner on coefficient fields 0..8 of the nx x nx log-normal workload (two
    right-hand sides each), every 4th, their scaled transforms cut into 64 x 64 crops of
    every shift (about n_target crops); Adam on the residual loss.  Field 9 is held out.
    (A second round on pairs from solves warm-started by the network was measured and
    dropped: over three seeds it left the 2048^2 warm-started solve at 150-208 FGMRES
    iterations with up to 45 rejected guesses, against 147-154 and none after the first
    round alone.)"""
    import torch
    from paper_2506_03947_amd import warmstart as W
    from synth import first_block_rhs, lognormal_kappa
    ny = nx
    kfn = lambda s: lognormal_kappa(nx, ny, 50.0, 10.0, 1.0, seed=1000 + s)  # noqa: E731
    rfn = lambda s: first_block_rhs(nx * ny, ell, seed=s)  # noqa: E731
    train_seeds, test_seed, b_seeds = list(range(9)), 9, (1, 2)
    lk = np.log(np.concatenate([kfn(s) for s in train_seeds[:2]]))
    c0, c1 = float(lk.mean()), float(lk.std())
    n_record, pick, crop = 60, 4, 64
    per_plane = max(1, n_target // (len(train_seeds) * len(b_seeds) * (n_record // pick) * (ell // 2 + 1)))
    t0 = time.perf_counter()
    train = W.generate_pairs(ctx, nx, ny, ell, alpha, kfn, train_seeds, rfn, b_seeds, n_record, pick, p_in, crop,
                             per_plane, c0, c1, restart=restart, log=None)
    held = W.generate_pairs(ctx, nx, ny, ell, alpha, kfn, [test_seed], rfn, b_seeds, n_record, pick, p_in, crop,
                            per_plane, c0, c1, seed=1, restart=restart, log=None)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    n_pairs = len(train)
    t0 = time.perf_counter()
    cnn, hist = W.train_network(ctx, train, steps, 64, 2e-3, 3, c0, c1, log=log, log_every=1000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    held_loss = W.eval_loss(ctx, cnn, held, 3)
    log(f"warm start: {n_pairs} pairs in {t_gen:.1f} s, training {t_train:.1f} s, held-out loss {held_loss:.3f}")
    record = {"grid": [nx, ny], "pairs": n_pairs, "gen_s": t_gen, "train_s": t_train, "adam_steps": steps,
              "first_loss": float(np.mean(hist[:20])), "final_loss": float(np.mean(hist[-100:])),
              "held_out_loss": held_loss, "held_out_field": test_seed}
    return cnn, record, kfn, rfn, test_seed


def warmstart_mode(a):
    """The learned warm start on its workload: 1024 x 1024, l = 10, alpha = 1e-2,
    kappa = 50 exp(g) (std 1, correlation 10 cells), p inner Chebyshev steps per shift,
    complex64 + bf16 kappa inner; the network trained by train_warm_start.  On the
    held-out field: solves to 1e-8 by FGMRES(restart) with the plain method in float64
    and in mixed precision, the network on every preconditioner input (cnn), on the first
    vector of each cycle (cnn_cycle), and as a minimal-residual correction before each
    cycle (cnn_mr, the headline value); and the plain mixed solve with FGMRES(7)."""
    from paper_2506_03947_amd import api
    from paper_2506_03947_amd import warmstart as W
    nx = ny = a.ws_nx
    ell, alpha, p_in = 10, 1e-2, a.p
    ctx = api.ac_ctx_create(0)
    cnn, trec, kfn, rfn, test_seed = train_warm_start(api, ctx, a.restart, p_in, a.ws_pairs, a.ws_steps, nx=nx)
    res = W.compare_solves(ctx, cnn, nx, ny, ell, alpha, kfn(test_seed), rfn(7), p_in, tol=a.tol, restart=a.restart,
                           reps=max(a.steps, 1), fp64_plain=True, modes=("plain", "cnn", "cnn_cycle", "cnn_mr"))
    r7 = W.compare_solves(ctx, cnn, nx, ny, ell, alpha, kfn(test_seed), rfn(7), p_in, tol=a.tol, restart=7,
                          reps=max(a.steps, 1), modes=("plain",))
    keep = ("outer_iters", "converged", "rel_residual_true", "cnn_fallbacks", "wall_s", "rel_diff_vs_fp64_plain")
    solves = {k: {f: v[f] for f in keep if f in v} for k, v in res.items() if k not in ("inner", "x")}
    solves["plain_restart7"] = {f: r7["plain"][f] for f in keep if f in r7["plain"]}
    for k, v in solves.items():
        log(f"{k}: {v}")
    t_ws = solves["cnn_mr"]["wall_s"]
    best_plain = min(solves["plain"]["wall_s"], solves["plain_restart7"]["wall_s"])
    print(json.dumps({
        "metric": "s per all-at-once solve to 1e-8 with the learned warm start (1024^2, l=10)", "value": t_ws,
        "warm_start_mode": "cnn_mr: minimal-residual correction along the warm-started P^-1 r before each cycle",
        "unit": "s/solve", "n_gpus": 1, "steps": max(a.steps, 1), "warmup": 1, "ms_per_step": 1000 * t_ws,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c64+bf16 (inner), f64 (outer)",
        "data": "synthetic",
        "config": {"workload": f"{nx}x{ny} log-normal kappa (kappa0 50, std 1, corr 10), l {ell}, alpha {alpha}, "
                               f"p {p_in}, FGMRES({a.restart}) to {a.tol}; network 5-16-16-2 3x3, bf16 weights"},
        "speedup_vs_plain_fp64": solves["plain_fp64"]["wall_s"] / t_ws,
        "speedup_vs_plain_mixed_same_restart": solves["plain"]["wall_s"] / t_ws,
        "speedup_vs_best_plain_mixed": best_plain / t_ws,
        "solves": solves, "inner_residual_per_shift": res["inner"], "training": trec,
    }), flush=True)


def kernels_only(a, api, prob, ell, n):
    """A few P_NC^{-1} applications in the solve's precision and launch shape, as many
    products with calA, then a plain device copy of known size (reference for the
    FETCH_SIZE/WRITE_SIZE scale)."""
    import torch
    L = api.L
    dev = torch.device("cuda:0")
    r = torch.randn(ell * n, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    opts = api.Opts(precision=L.AC_PREC_MIXED_BF16K, p=a.p)
    ws = api.workspace(api.ac_prec_workspace_size(prob, opts))
    ctx = prob.ctx
    api.ac_apply_prec(prob, opts, r, z, ws)
    api.ac_ctx_set_profiling(ctx, True)
    api.ac_ctx_reset_stats(ctx)
    for _ in range(max(a.steps, 1)):
        api.ac_apply_prec(prob, opts, r, z, ws)
    for _ in range(max(a.steps, 1)):
        api.ac_apply_A(prob, r, z)
    stats = api.ac_ctx_kernel_stats(ctx)
    api.ac_ctx_set_profiling(ctx, False)
    out_ceil = stream_ceilings(api, ctx)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)  # 512 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    out = {"mode": "kernels", "copy_bytes_each_way": src.numel() * 8, "stream_ceilings_GBps": out_ceil}
    for name in ("cheb_step", "cheb_pair", "cheb_triple", "apply_calA"):
        st = stats[name]
        if st["launches"]:
            avg_ms = st["ms"] / st["launches"]
            per = st["bytes"] / st["launches"]
            out[name] = {"avg_ms": avg_ms, "bytes_per_launch": per, "GBps": per / avg_ms / 1e6,
                         "launches": st["launches"]}
    print(json.dumps(out), flush=True)


def stream_ceilings(api, ctx, bytes_total=5 * 512 * 1024 * 1024):
    """GB/s of the library's pure streaming kernel for a few read / write mixes."""
    ws = api.workspace(bytes_total)
    out = {}
    for name, (r, w) in (("read", (1, 0)), ("copy", (1, 1)), ("triad", (2, 1)), ("3R2W", (3, 2))):
        out[name] = api.ac_stream_bandwidth(ctx, r, w, ws, reps=20)
    del ws
    log(f"stream ceilings GB/s: {out}")
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(a, name, sources):
    """HBM bytes per launch of the roofline kernel from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record (scaled by a copy of known size), or None when the record does not
    cover this workload or a kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if a.workload != "large" or a.p != 20 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2506_03947_amd", "csrc", f), "rb").read())
    if h.hexdigest() != rec["kernel_source_sha256"]:
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(w, kappa, b, p, restart, gpu_outer_iters):
    """The oracle (numpy/scipy float64) timed on the host on a bounded sample of the same
    workload, scaled to the metric's unit (s per solve) by the GPU's outer-iteration count.

    oracle-MT (the reported value): one complete FGMRES(restart) cycle of the oracle --
    restart iterations, each one P_NC^{-1} application (all l shifts, p Chebyshev steps,
    sparse complex128, the shifted solves on a thread pool), one calA product and CGS2
    against the basis so far -- plus the cycle's solution update and true residual.
    oracle-1T: the first iteration of the same cycle with the shifted solves one after
    another on one thread (scipy CSR products and numpy's FFT are single-threaded)."""
    from oracle import operators as ops
    from oracle import precond as pc
    from oracle.krylov import fgmres
    nx, ny, ell, alpha = w["nx"], w["ny"], w["ell"], w["alpha"]
    A = ops.build_A(2, nx, ny, kappa)
    lo, hi = ops.spectral_interval(2, nx, ny, kappa)
    cpus = len(os.sched_getaffinity(0))
    workers = max(1, min(ell, cpus))
    op = lambda v: ops.apply_calA(A, v, ell)

    def timed(nw, its):
        t0 = time.perf_counter()
        _, inf = fgmres(op, b, lambda v: pc.apply_prec_nc(A, v, ell, alpha, lo, hi, p, workers=nw), tol=0.0,
                        m=restart, max_outer=its)
        return time.perf_counter() - t0, inf["iterations"]

    t_mt, it_mt = timed(workers, restart)
    log(f"oracle-MT: {it_mt} FGMRES iterations in {t_mt:.2f} s on {workers} threads")
    t_1t, it_1t = timed(1, 1)
    log(f"oracle-1T: {it_1t} FGMRES iteration in {t_1t:.2f} s")
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    scale = max(gpu_outer_iters, 1)
    return {
        "value": t_mt / it_mt * scale,
        "unit": "s/solve",
        "cores": workers,
        "kind": "oracle",
        "sample": (f"one full oracle FGMRES({restart}) cycle at {nx}x{ny} (l={ell}, p={p}; {it_mt} iterations, "
                   f"each P_NC^-1 with the l shifted solves on {workers} threads, calA, CGS2; plus the update and "
                   f"true residual) timed {t_mt:.2f} s, scaled by the GPU's {gpu_outer_iters} outer iterations"),
        "oracle_1T": {"value": t_1t / it_1t * scale, "cores": 1,
                      "sample": f"the first iteration of the same cycle on one thread, timed {t_1t:.2f} s, scaled "
                                f"by {gpu_outer_iters} iterations"},
        "host_cpus_visible": cpus,
        "cpu_model": cpu_model,
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    if a.mode == "batch":
        batch_mode(a)
        return
    if a.mode == "exact":
        exact_mode(a)
        return
    if a.mode == "sp":
        sp_mode(a)
        return
    if a.mode == "blocks":
        blocks_mode(a)
        return
    if a.mode == "paper":
        paper_mode(a)
        return
    if a.mode == "warmstart":
        warmstart_mode(a)
        return
    import torch
    from paper_2506_03947_amd import api
    from synth import lognormal_kappa, first_block_rhs
    L = api.L

    w = WORKLOADS[a.workload]
    nx, ny, ell, alpha = w["nx"], w["ny"], w["ell"], w["alpha"]
    n = nx * ny
    log(f"inputs {nx}x{ny} l={ell}")
    kappa = lognormal_kappa(nx, ny, w["kappa0"], w["corr"], w["std"], seed=a.seed)
    b = first_block_rhs(n, ell, seed=a.seed)
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(kappa).to(dev)
    bd = torch.from_numpy(b).to(dev)
    x = torch.zeros(ell * n, dtype=torch.float64, device=dev)
    ctx = api.ac_ctx_create(0)
    api.ac_ctx_set_step_pairs(ctx, a.step_pairs, *a.pair_tiling)
    api.ac_ctx_set_step_triples(ctx, a.step_triples, *a.triple_tiling)
    prob = api.ac_problem_create(ctx, 2, nx, ny, kd, ell, alpha)
    mu_lo, mu_hi = api.ac_spectral_bounds(prob)
    if a.mode == "kernels":
        kernels_only(a, api, prob, ell, n)
        return

    def run(precision, steps, warmup, profile):
        opts = api.Opts(precision=precision, p=a.p, tol=a.tol, restart_m=a.restart, max_outer=3000)
        ws = api.workspace(api.ac_solve_workspace_size(prob, opts))
        info = None
        for i in range(warmup):
            x.zero_()
            info = api.ac_solve(prob, opts, bd, x, ws)
            log(f"warmup {i} prec={precision} iters={info['outer_iters']} res={info['rel_residual_true']:.2e} "
                f"t={info['seconds']:.3f}s")
        api.ac_ctx_set_profiling(ctx, profile)
        api.ac_ctx_reset_stats(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for i in range(steps):
            x.zero_()
            infos.append(api.ac_solve(prob, opts, bd, x, ws))
            log(f"step {i} prec={precision} iters={infos[-1]['outer_iters']} "
                f"res={infos[-1]['rel_residual_true']:.2e} t={infos[-1]['seconds']:.3f}s")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = api.ac_ctx_kernel_stats(ctx)
        api.ac_ctx_set_profiling(ctx, False)
        xs = x.clone()
        del ws
        return dt / steps, infos[-1], stats, xs

    prec_mixed = L.AC_PREC_MIXED_BF16K
    t_mixed, info_mixed, stats_mixed, x_mixed = run(prec_mixed, a.steps, a.warmup, True)
    out_fp64 = None
    if not a.no_fp64:
        t64, info64, stats64, x64 = run(L.AC_PREC_FP64, max(1, a.steps // 2), 1, True)
        diff = float(torch.linalg.norm(x_mixed - x64) / torch.linalg.norm(x64))
        out_fp64 = {"s_per_solve": t64, "outer_iters": info64["outer_iters"],
                    "rel_residual_true": info64["rel_residual_true"],
                    # steady Chebyshev steps (blocks of three, pairs, single sweeps): unfused
                    # algorithmic bytes per second over all of them
                    "steady_steps_GBps": sum(stats64[k]["bytes"] for k in ("cheb_triple", "cheb_pair", "cheb_step")) /
                    max(sum(stats64[k]["ms"] for k in ("cheb_triple", "cheb_pair", "cheb_step")), 1e-9) / 1e6,
                    "speedup_mixed_vs_fp64": t64 / t_mixed,
                    "mixed_vs_fp64_solution_rel_diff": diff}

    # Dominant kernel: the steady-sweep class with the most time per solve (fused blocks of
    # three steps, pairs, or single sweeps).  The library counts each launch's own minimum
    # HBM bytes: every operand stream it must read or write once (a block of three steps:
    # x_k, x_{k-1}, rhat in, x_{k+2}, x_{k+3} out per computing shift, kappa once per launch).
    # `achieved` = those bytes / the average launch time (HIP events on the library's
    # stream); `effective_GBps` restates the same time against the bytes the same steps
    # would move as unfused single sweeps (4 streams per shift and step, kappa per step),
    # which a fused block beats by construction and so is never a fraction of the peak.
    kinds = {
        "cheb_triple": (3, "cheb_triple_kernel (complex64 iterates, bf16 kappa, 2 points per lane): three steady "
                           "shifted-Chebyshev steps fused in one sweep",
                        "cheb_triple_2048x2048_l10_traffic.json", TRIPLE_SOURCES),
        "cheb_pair": (2, "cheb_pair_kernel: two steady shifted-Chebyshev steps fused in one sweep", None, None),
        "cheb_step": (1, "cheb_sweep_kernel: steady-state shifted Chebyshev sweep", None, None),
    }
    dom = max((k for k in kinds if stats_mixed[k]["launches"]), key=lambda k: stats_mixed[k]["ms"])
    depth, kname, tfile, tsrc = kinds[dom]
    st = stats_mixed[dom]
    traffic = measured_traffic(a, tfile, tsrc) if tfile else None
    avg_ms = st["ms"] / max(st["launches"], 1)
    bytes_per_launch = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    nsr = 2 if ell % 2 == 0 else 1
    nsc = (ell - nsr) // 2
    per_stream = 4.0 * nsr + 8.0 * nsc  # bytes of one complex64 / float32 stream over all shifts, per point
    roofline = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": bytes_per_launch,
                "launches": st["launches"], "steps_per_launch": depth}
    if dom == "cheb_triple":
        # steady blocks per application from a zero guess: steps 1..3 are the first block,
        # the last step is fused with the inverse transform, steps 4..p-2 are cut into threes
        blocks = a.steps * info_mixed["outer_iters"] * ((a.p - 5) // 3)
        unfused = blocks * n * 3 * (4.0 * per_stream + 2.0)
        roofline["effective_GBps"] = unfused / (st["ms"] * 1e-3) / 1e9
        if traffic:
            roofline["traffic_GBps"] = traffic / (avg_ms * 1e-3) / 1e9
            roofline["traffic_frac"] = roofline["traffic_GBps"] / HBM_PEAK_GBS
            roofline["traffic_over_own_min"] = traffic / bytes_per_launch
        roofline["note"] = ("achieved = the launch's own minimum bytes (every operand stream once) / time; "
                            "traffic = rocprofv3 FETCH_SIZE + WRITE_SIZE per launch (scaled by a copy of known "
                            "size); effective_GBps = the unfused single-step bytes of the same steps / the same "
                            "time (not a bandwidth)")

    # streaming ceilings of this GPU for the read / write mixes in question (a kernel that
    # only moves its streams): read-only, copy, triad, and the fused block's 3 reads + 2
    # writes
    ceilings = stream_ceilings(api, ctx)
    roofline["stream_ceilings_GBps"] = ceilings
    roofline["frac_of_stream_ceiling"] = achieved / ceilings["3R2W"]

    # the other inner budgets of the workload (p = 5, 10): same solve, fewer steps per shift
    budgets = {}
    if not a.no_budgets:
        for pb in (5, 10):
            if pb == a.p:
                continue
            opts = api.Opts(precision=prec_mixed, p=pb, tol=a.tol, restart_m=a.restart, max_outer=3000)
            ws = api.workspace(api.ac_solve_workspace_size(prob, opts))
            x.zero_()
            api.ac_solve(prob, opts, bd, x, ws)
            ts = []
            for _ in range(2):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                inf = api.ac_solve(prob, opts, bd, x, ws)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            budgets[f"p{pb}"] = {"s_per_solve": min(ts), "outer_iters": inf["outer_iters"],
                                 "converged": inf["converged"], "rel_residual_true": inf["rel_residual_true"]}
            log(f"budget p={pb}: {budgets[f'p{pb}']}")
            del ws

    # oracle checks of the results: the true residual of the headline (mixed) solution
    # recomputed on the host by the oracle's calA, and the same solve with a constant
    # coefficient (kappa0, exact in bfloat16) against the oracle's closed-form sequential
    # chain (sine transform, Appendix A), in mixed and float64 inner precision
    from oracle import operators as ops
    A_host = ops.build_A(2, nx, ny, kappa)
    xm = x_mixed.cpu().numpy()
    rel_res_oracle = float(np.linalg.norm(b - ops.apply_calA(A_host, xm, ell)) / np.linalg.norm(b))
    del A_host, xm
    const = {}
    if not a.no_const_check:
        kc = torch.full((n,), w["kappa0"], dtype=torch.float64, device=dev)
        pc_ = api.ac_problem_create(ctx, 2, nx, ny, kc, ell, alpha)
        x_ref = ops.sequential_solve_closed_form(2, nx, ny, w["kappa0"], b, ell)
        ref_norm = np.linalg.norm(x_ref)
        for name, pr in (("mixed", prec_mixed), ("fp64", L.AC_PREC_FP64)):
            opts = api.Opts(precision=pr, p=a.p, tol=a.tol, restart_m=a.restart, max_outer=3000)
            ws = api.workspace(api.ac_solve_workspace_size(pc_, opts))
            x.zero_()
            api.ac_solve(pc_, opts, bd, x, ws)
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            inf = api.ac_solve(pc_, opts, bd, x, ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float(np.linalg.norm(x.cpu().numpy() - x_ref) / ref_norm)
            const[name] = {"s_per_solve": dt, "outer_iters": inf["outer_iters"],
                           "rel_residual_true": inf["rel_residual_true"], "rel_err_vs_oracle": err}
            log(f"constant kappa {name}: {const[name]}")
            del ws
        del pc_, kc, x_ref

    # the learned warm start on the same problem: the network trained on the 1024^2
    # workload (train_warm_start), applied as a minimal-residual correction before each
    # FGMRES cycle (AC_INNER_CHEB_CNN_MR), mixed precision; against the plain method in
    # float64 and mixed precision above
    warm = None
    if not a.no_warm_start:
        net, trec, _, _, _ = train_warm_start(api, ctx, a.restart, a.p, a.ws_pairs, a.ws_steps)
        api.ac_problem_attach_cnn(prob, net)
        opts = api.Opts(precision=prec_mixed, inner=L.AC_INNER_CHEB_CNN_MR, p=a.p, tol=a.tol, restart_m=a.restart,
                        max_outer=3000)
        ws = api.workspace(api.ac_solve_workspace_size(prob, opts))
        x.zero_()
        api.ac_solve(prob, opts, bd, x, ws)
        ts = []
        for _ in range(max(2, a.steps // 4)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            inf = api.ac_solve(prob, opts, bd, x, ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t_w = sum(ts) / len(ts)
        warm = {"mode": "minimal-residual correction along the warm-started P^-1 r before each FGMRES cycle",
                "s_per_solve": t_w, "outer_iters": inf["outer_iters"], "restarts": inf["restarts"],
                "matvecs_A": inf["matvecs_A"], "cnn_fallbacks": inf["cnn_fallbacks"],
                "rel_residual_true": inf["rel_residual_true"],
                "speedup_vs_plain_mixed": t_mixed / t_w,
                "speedup_vs_plain_fp64": (out_fp64["s_per_solve"] / t_w) if out_fp64 else None,
                "rel_diff_vs_fp64_solution": (float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
                                              if out_fp64 else None),
                "training": trec}
        log(f"warm start: {warm['s_per_solve']:.3f} s, {warm['outer_iters']} iterations")
        del ws
        api.ac_problem_attach_cnn(prob, None)

    cpu = None
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(w, kappa, b, a.p, a.restart, info_mixed["outer_iters"])

    kernels = {k: {"ms_per_solve": v["ms"] / a.steps, "launches_per_solve": v["launches"] / a.steps,
                   "GBps": (v["bytes"] / v["ms"] / 1e6) if v["ms"] > 0 else None}
               for k, v in stats_mixed.items() if v["launches"]}
    res = {
        "metric": "s per all-at-once solve to 1e-8 + shifted-stencil GB/s (% HBM peak), mixed vs FP64",
        "value": t_mixed,
        "unit": "s/solve",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+bf16 (inner), f64 (outer)",
        "data": "synthetic",
        "config": {"workload": (f"2D {nx}x{ny} log-normal kappa (kappa0={w['kappa0']}, std={w['std']}, "
                                f"corr={w['corr']} cells), l={ell}, alpha={alpha}, p={a.p}, FGMRES({a.restart}) "
                                f"to {a.tol}"),
                   "nx": nx, "ny": ny, "ell": ell, "alpha": alpha, "p": a.p, "restart": a.restart,
                   "tol": a.tol, "mu_lo": mu_lo, "mu_hi": mu_hi},
        "outer_iters": info_mixed["outer_iters"],
        "rel_residual_true": info_mixed["rel_residual_true"],
        "rel_residual_oracle": rel_res_oracle,
        "matvecs_A": info_mixed["matvecs_A"],
        "orth_loss": info_mixed["orth_loss"],
        "shifted_stencil_GBps": achieved,
        "shifted_stencil_pct_hbm_peak": 100 * achieved / HBM_PEAK_GBS,
        "fp64": out_fp64,
        "budgets": budgets,
        "constant_kappa_check": const,
        "warm_start": warm,
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
