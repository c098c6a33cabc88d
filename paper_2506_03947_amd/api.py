"""Python binding of the alphacirc C ABI: same names, argument marshalling only.

Device buffers are torch tensors on the GPU (float64 block vectors of length
l*N, layout x[k*N + i]); their data pointers go straight to the library, which
runs every step in its HIP kernels on the context's stream.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from ._lib import check


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _f64(t: torch.Tensor, n: int, name: str):
    if t.dtype != torch.float64 or t.numel() != n:
        raise ValueError(f"{name}: expected {n} float64 values, got {t.numel()} {t.dtype}")
    return _ptr(t)


class Ctx:
    def __init__(self, handle, device, stream):
        self.h = handle
        self.device = device
        self.stream = stream

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L._lib is not None:
            L._lib.ac_ctx_destroy(self.h)
        self.h = None


class Problem:
    def __init__(self, handle, ctx, n, ell, ns):
        self.h = handle
        self.ctx = ctx
        self.n = n
        self.ell = ell
        self.ns = ns

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L._lib is not None:
            L._lib.ac_problem_destroy(self.h)
        self.h = None


@dataclass
class Opts:
    precision: int = L.AC_PREC_FP64
    inner: int = L.AC_INNER_CHEB
    p: object = 10          # int (uniform) or a length-l sequence
    tol: float = 1e-8
    restart_m: int = 30
    max_outer: int = 500
    outer: int = L.AC_OUTER_FGMRES

    def to_c(self, ell: int):
        o = L.ac_solve_opts()
        o.precision = self.precision
        o.inner = self.inner
        if isinstance(self.p, int):
            o.p_uniform = int(self.p)
            o.p_per_shift = None
            keep = None
        else:
            arr = (C.c_int * ell)(*[int(v) for v in self.p])
            o.p_per_shift = C.cast(arr, C.POINTER(C.c_int))
            o.p_uniform = 0
            keep = arr
        o.tol = float(self.tol)
        o.restart_m = int(self.restart_m)
        o.max_outer = int(self.max_outer)
        o.outer = int(self.outer)
        return o, keep


def ac_status_string(status: int) -> str:
    return L.load().ac_status_string(status).decode()


def ac_last_error() -> str:
    return L.load().ac_last_error().decode()


def ac_ctx_create(device: int = 0, stream: torch.cuda.Stream | None = None) -> Ctx:
    lib = L.load()
    stream = stream if stream is not None else torch.cuda.current_stream(device)
    h = C.c_void_p()
    check(lib.ac_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)), "ac_ctx_create")
    return Ctx(h, device, stream)


def ac_ctx_set_profiling(ctx: Ctx, on: bool) -> None:
    check(L.load().ac_ctx_set_profiling(ctx.h, int(bool(on))), "ac_ctx_set_profiling")


def ac_ctx_kernel_stats(ctx: Ctx) -> dict:
    ms = (C.c_double * L.AC_K_COUNT)()
    launches = (C.c_longlong * L.AC_K_COUNT)()
    nbytes = (C.c_double * L.AC_K_COUNT)()
    check(L.load().ac_ctx_kernel_stats(ctx.h, ms, launches, nbytes), "ac_ctx_kernel_stats")
    return {name: {"ms": ms[i], "launches": launches[i], "bytes": nbytes[i]}
            for i, name in enumerate(L.KERNEL_CLASS_NAMES)}


def ac_ctx_reset_stats(ctx: Ctx) -> None:
    check(L.load().ac_ctx_reset_stats(ctx.h), "ac_ctx_reset_stats")


def ac_ctx_set_tiling(ctx: Ctx, rows_per_wave: int = 0, waves_per_block: int = 0, points_per_lane: int = 0) -> None:
    check(L.load().ac_ctx_set_tiling(ctx.h, rows_per_wave, waves_per_block, points_per_lane), "ac_ctx_set_tiling")


def ac_problem_create(ctx: Ctx, dim: int, nx: int, ny: int, kappa: torch.Tensor, ell: int, alpha: float,
                      bc: int = L.AC_BC_DIRICHLET, bounds: tuple[float, float] | None = None) -> Problem:
    lib = L.load()
    g = L.ac_grid(dim, nx, ny, bc)
    n = nx * ny
    kp = _f64(kappa, n, "kappa")
    bp = None
    if bounds is not None:
        bp = C.byref(L.ac_bounds(float(bounds[0]), float(bounds[1])))
    h = C.c_void_p()
    check(lib.ac_problem_create(ctx.h, C.byref(g), kp, ell, float(alpha), bp, C.byref(h)), "ac_problem_create")
    nn, ee, ns = C.c_longlong(), C.c_int(), C.c_int()
    check(lib.ac_problem_dims(h, C.byref(nn), C.byref(ee), C.byref(ns)), "ac_problem_dims")
    return Problem(h, ctx, nn.value, ee.value, ns.value)


def ac_problem_create_blocks(ctx: Ctx, dim: int, nx: int, ny: int, kappa_blocks: torch.Tensor, ell: int,
                             alpha: float, bc: int = L.AC_BC_DIRICHLET,
                             bounds: tuple[float, float] | None = None) -> Problem:
    """Varying diagonal blocks: kappa_blocks holds l coefficient fields (l * N float64)."""
    lib = L.load()
    g = L.ac_grid(dim, nx, ny, bc)
    kp = _f64(kappa_blocks, ell * nx * ny, "kappa_blocks")
    bp = C.byref(L.ac_bounds(float(bounds[0]), float(bounds[1]))) if bounds is not None else None
    h = C.c_void_p()
    check(lib.ac_problem_create_blocks(ctx.h, C.byref(g), kp, ell, float(alpha), bp, C.byref(h)),
          "ac_problem_create_blocks")
    nn, ee, ns = C.c_longlong(), C.c_int(), C.c_int()
    check(lib.ac_problem_dims(h, C.byref(nn), C.byref(ee), C.byref(ns)), "ac_problem_dims")
    return Problem(h, ctx, nn.value, ee.value, ns.value)


def ac_spectral_bounds(p: Problem) -> tuple[float, float]:
    lo, hi = C.c_double(), C.c_double()
    check(L.load().ac_spectral_bounds(p.h, C.byref(lo), C.byref(hi)), "ac_spectral_bounds")
    return lo.value, hi.value


def ac_problem_shifts(p: Problem):
    """lambda_m, m = 0..l-1, as a complex numpy array."""
    import numpy as np
    buf = (C.c_double * (2 * p.ell))()
    check(L.load().ac_problem_shifts(p.h, buf), "ac_problem_shifts")
    v = np.frombuffer(buf, dtype=np.float64).copy()
    return v[0::2] + 1j * v[1::2]


def ac_alloc_nc2(p: Problem, budget: float) -> list[int]:
    out = (C.c_int * p.ell)()
    check(L.load().ac_alloc_nc2(p.h, float(budget), out), "ac_alloc_nc2")
    return list(out)


def ac_alloc_nc1(p: Problem, budget: float) -> list[int]:
    out = (C.c_int * p.ell)()
    check(L.load().ac_alloc_nc1(p.h, float(budget), out), "ac_alloc_nc1")
    return list(out)


def ac_prec_workspace_size(p: Problem, opts: Opts) -> int:
    o, keep = opts.to_c(p.ell)
    n = C.c_size_t()
    check(L.load().ac_prec_workspace_size(p.h, C.byref(o), C.byref(n)), "ac_prec_workspace_size")
    return n.value


def ac_solve_workspace_size(p: Problem, opts: Opts) -> int:
    o, keep = opts.to_c(p.ell)
    n = C.c_size_t()
    check(L.load().ac_solve_workspace_size(p.h, C.byref(o), C.byref(n)), "ac_solve_workspace_size")
    return n.value


def workspace(nbytes: int, device: int = 0) -> torch.Tensor:
    """A device byte buffer to pass as workspace."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{device}")


def ac_apply_A(p: Problem, x: torch.Tensor, y: torch.Tensor) -> None:
    n = p.ell * p.n
    check(L.load().ac_apply_A(p.h, _f64(x, n, "x"), _f64(y, n, "y")), "ac_apply_A")


def ac_apply_prec(p: Problem, opts: Opts, r: torch.Tensor, z: torch.Tensor, ws: torch.Tensor) -> None:
    n = p.ell * p.n
    o, keep = opts.to_c(p.ell)
    check(L.load().ac_apply_prec(p.h, C.byref(o), _f64(r, n, "r"), _f64(z, n, "z"), _ptr(ws), ws.numel()),
          "ac_apply_prec")


def ac_apply_prec_noalloc(p: Problem, opts: Opts, r: torch.Tensor, z: torch.Tensor) -> None:
    """ac_apply_prec with the library's fixed device scratch as workspace (no allocation)."""
    n = p.ell * p.n
    o, keep = opts.to_c(p.ell)
    check(L.load().ac_apply_prec_noalloc(p.h, C.byref(o), _f64(r, n, "r"), _f64(z, n, "z")),
          "ac_apply_prec_noalloc")
    del keep


def ac_stream_bandwidth(ctx: Ctx, reads: int, writes: int, ws: torch.Tensor, reps: int = 20) -> float:
    """GB/s of a kernel that only streams `reads` inputs and `writes` outputs (calibration)."""
    out = C.c_double()
    check(L.load().ac_stream_bandwidth(ctx.h, int(reads), int(writes), _ptr(ws), ws.numel(), int(reps),
                                       C.byref(out)), "ac_stream_bandwidth")
    return out.value


def ac_spectral_offsets(p: Problem, precision: int) -> list[int]:
    off = (C.c_longlong * (p.ns + 1))()
    check(L.load().ac_spectral_offsets(p.h, precision, off), "ac_spectral_offsets")
    return list(off)


def spectral_dtype(precision: int) -> torch.dtype:
    return torch.float64 if precision == L.AC_PREC_FP64 else torch.float32


def ac_tdft_forward(p: Problem, precision: int, r: torch.Tensor, rhat: torch.Tensor) -> None:
    check(L.load().ac_tdft_forward(p.h, precision, _f64(r, p.ell * p.n, "r"), _ptr(rhat)), "ac_tdft_forward")


def ac_shifted_cheb(p: Problem, opts: Opts, rhat: torch.Tensor, x0hat: torch.Tensor | None, yhat: torch.Tensor,
                    ws: torch.Tensor) -> None:
    o, keep = opts.to_c(p.ell)
    check(L.load().ac_shifted_cheb(p.h, C.byref(o), _ptr(rhat), _ptr(x0hat), _ptr(yhat), _ptr(ws), ws.numel()),
          "ac_shifted_cheb")


def ac_tdft_inverse(p: Problem, precision: int, yhat: torch.Tensor, z: torch.Tensor) -> None:
    check(L.load().ac_tdft_inverse(p.h, precision, _ptr(yhat), _f64(z, p.ell * p.n, "z")), "ac_tdft_inverse")


def ac_solve(p: Problem, opts: Opts, b: torch.Tensor, x: torch.Tensor, ws: torch.Tensor) -> dict:
    n = p.ell * p.n
    o, keep = opts.to_c(p.ell)
    info = L.ac_solve_info()
    st = check(L.load().ac_solve(p.h, C.byref(o), _f64(b, n, "b"), _f64(x, n, "x"), _ptr(ws), ws.numel(),
                                 C.byref(info)), "ac_solve")
    return _info_dict(st, info)


def ac_solve_record(p: Problem, opts: Opts, b: torch.Tensor, x: torch.Tensor, ws: torch.Tensor,
                    rec: torch.Tensor) -> tuple[dict, int]:
    """ac_solve that copies the first rec.shape[0] preconditioner inputs into rec
    ([count, l*N] float64); returns (info, number recorded)."""
    n = p.ell * p.n
    o, keep = opts.to_c(p.ell)
    info = L.ac_solve_info()
    done = C.c_int()
    count = rec.shape[0]
    st = check(L.load().ac_solve_record(p.h, C.byref(o), _f64(b, n, "b"), _f64(x, n, "x"), _ptr(ws), ws.numel(),
                                        C.byref(info), _f64(rec, count * n, "rec"), count, C.byref(done)),
               "ac_solve_record")
    return _info_dict(st, info), done.value


def _handles(items):
    arr = (C.c_void_p * len(items))()
    for i, h in enumerate(items):
        arr[i] = h.value if isinstance(h, C.c_void_p) else h
    return arr


def ac_ctx_set_shift_groups(ctx: Ctx, mode: int) -> None:
    check(L.load().ac_ctx_set_shift_groups(ctx.h, int(mode)), "ac_ctx_set_shift_groups")


def ac_ctx_set_step_triples(ctx: Ctx, mode: int, rows_per_wave: int = 0, waves_per_simd: int = 0,
                            points_per_lane: int = 0) -> None:
    check(L.load().ac_ctx_set_step_triples(ctx.h, int(mode), int(rows_per_wave), int(waves_per_simd),
                                           int(points_per_lane)), "ac_ctx_set_step_triples")


def ac_ctx_set_step_pairs(ctx: Ctx, mode: int, rows_per_wave: int = 0, waves_per_block: int = 0,
                          points_per_lane: int = 0) -> None:
    check(L.load().ac_ctx_set_step_pairs(ctx.h, int(mode), int(rows_per_wave), int(waves_per_block),
                                         int(points_per_lane)), "ac_ctx_set_step_pairs")


def ac_problem_set_tiling(p: Problem, rows_per_wave: int = 0, waves_per_block: int = 0,
                          points_per_lane: int = 0) -> None:
    check(L.load().ac_problem_set_tiling(p.h, rows_per_wave, waves_per_block, points_per_lane),
          "ac_problem_set_tiling")


def ac_tune_tiling(p: Problem, precision: int, ws: torch.Tensor, cache_path: str | None = None) -> tuple[list, float]:
    """Tunes p's sweep tiling; returns ([rows per wave, waves per block, points per
    lane], microseconds per sweep or 0.0 when read from the cache)."""
    out = (C.c_int * 3)()
    us = C.c_double()
    check(L.load().ac_tune_tiling(p.h, precision, cache_path.encode() if cache_path else None, _ptr(ws), ws.numel(),
                                  out, C.byref(us)), "ac_tune_tiling")
    return list(out), us.value


def ac_batch_workspace_size(ctx: Ctx, problems: list, opts: Opts) -> int:
    o, keep = opts.to_c(problems[0].ell)
    n = C.c_size_t()
    check(L.load().ac_batch_workspace_size(ctx.h, len(problems), _handles([p.h for p in problems]), C.byref(o),
                                           C.byref(n)), "ac_batch_workspace_size")
    return n.value


def ac_batch_solve(ctx: Ctx, problems: list, opts: Opts, bs: list, xs: list, ws: torch.Tensor) -> list[dict]:
    """Solves every problem (device b, x tensors) in one batched run; returns the
    per-problem info dicts."""
    k = len(problems)
    o, keep = opts.to_c(problems[0].ell)
    bp = _handles([_f64(b, p.ell * p.n, "b") for b, p in zip(bs, problems)])
    xp = _handles([_f64(x, p.ell * p.n, "x") for x, p in zip(xs, problems)])
    infos = (L.ac_solve_info * k)()
    st = check(L.load().ac_batch_solve(ctx.h, k, _handles([p.h for p in problems]), C.byref(o), bp, xp, _ptr(ws),
                                       ws.numel(), infos), "ac_batch_solve")
    return [_info_dict(st, infos[i]) for i in range(k)]


def _info_dict(st, info) -> dict:
    return {
        "status": st,
        "converged": st == L.AC_OK,
        "outer_iters": info.outer_iters,
        "restarts": info.restarts,
        "matvecs_A": info.matvecs_A,
        "rel_residual_true": info.rel_residual_true,
        "seconds": info.seconds,
        "cnn_fallbacks": info.cnn_fallbacks,
        "orth_loss": info.orth_loss,
    }


# ---- spectral buffer helpers (host side views, no arithmetic) -------------------

def spectral_to_complex(p: Problem, precision: int, buf: torch.Tensor):
    """Split a spectral buffer into per-frequency complex tensors (m = 0..l_s-1)."""
    off = ac_spectral_offsets(p, precision)
    out = []
    for m in range(p.ns):
        real = (m == 0) or (p.ell % 2 == 0 and m == p.ell // 2)
        sl = buf[off[m]: off[m] + (p.n if real else 2 * p.n)]
        if real:
            out.append(torch.complex(sl, torch.zeros_like(sl)))
        else:
            v = sl.view(p.n, 2)
            out.append(torch.complex(v[:, 0].contiguous(), v[:, 1].contiguous()))
    return out


def complex_to_spectral(p: Problem, precision: int, slices) -> torch.Tensor:
    """Pack per-frequency complex tensors (m = 0..l_s-1) into a spectral buffer."""
    off = ac_spectral_offsets(p, precision)
    dt = spectral_dtype(precision)
    dev = slices[0].device
    buf = torch.zeros(off[-1], dtype=dt, device=dev)
    for m in range(p.ns):
        real = (m == 0) or (p.ell % 2 == 0 and m == p.ell // 2)
        s = slices[m]
        if real:
            buf[off[m]: off[m] + p.n] = s.real.to(dt)
        else:
            buf[off[m]: off[m] + 2 * p.n] = torch.stack([s.real, s.imag], dim=1).reshape(-1).to(dt)
    return buf


# ---- learned warm start ---------------------------------------------------------------

class Cnn:
    def __init__(self, handle, ctx):
        self.h = handle
        self.ctx = ctx

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L._lib is not None:
            L._lib.ac_cnn_destroy(self.h)
        self.h = None


def ac_cnn_param_count() -> int:
    return L.load().ac_cnn_param_count()


def ac_cnn_create(ctx: Ctx) -> Cnn:
    h = C.c_void_p()
    check(L.load().ac_cnn_create(ctx.h, C.byref(h)), "ac_cnn_create")
    return Cnn(h, ctx)


def ac_cnn_set_params(cnn: Cnn, params, c0: float, c1: float) -> None:
    import numpy as np
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
    if p.size != ac_cnn_param_count():
        raise ValueError(f"expected {ac_cnn_param_count()} parameters, got {p.size}")
    check(L.load().ac_cnn_set_params(cnn.h, p.ctypes.data_as(C.POINTER(C.c_float)), float(c0), float(c1)),
          "ac_cnn_set_params")


def ac_cnn_get_params(cnn: Cnn):
    import numpy as np
    p = np.empty(ac_cnn_param_count(), dtype=np.float32)
    c0, c1 = C.c_double(), C.c_double()
    check(L.load().ac_cnn_get_params(cnn.h, p.ctypes.data_as(C.POINTER(C.c_float)), C.byref(c0), C.byref(c1)),
          "ac_cnn_get_params")
    return p, c0.value, c1.value


def ac_cnn_workspace_size(batch: int, height: int, width: int) -> int:
    n = C.c_size_t()
    check(L.load().ac_cnn_workspace_size(batch, height, width, C.byref(n)), "ac_cnn_workspace_size")
    return n.value


def _u16(t: torch.Tensor, n: int, name: str):
    if t.dtype not in (torch.int16, torch.uint16) or t.numel() != n:
        raise ValueError(f"{name}: expected {n} 16-bit values, got {t.numel()} {t.dtype}")
    return _ptr(t)


def _f32(t: torch.Tensor, n: int, name: str):
    if t.dtype != torch.float32 or t.numel() != n:
        raise ValueError(f"{name}: expected {n} float32 values, got {t.numel()} {t.dtype}")
    return _ptr(t)


def ac_cnn_forward(cnn: Cnn, x: torch.Tensor, batch: int, height: int, width: int, y: torch.Tensor,
                   ws: torch.Tensor) -> None:
    npx = batch * height * width
    check(L.load().ac_cnn_forward(cnn.h, _u16(x, npx * 16, "x"), batch, height, width, _f32(y, npx * 2, "y"),
                                  _ptr(ws), ws.numel()), "ac_cnn_forward")


def ac_cnn_grad(cnn: Cnn, x: torch.Tensor, t: torch.Tensor, tnorm: torch.Tensor, border: int, batch: int,
                height: int, width: int, ws: torch.Tensor, want_grad: bool = False):
    import numpy as np
    npx = batch * height * width
    loss = C.c_double()
    g = np.empty(ac_cnn_param_count(), dtype=np.float32) if want_grad else None
    check(L.load().ac_cnn_grad(cnn.h, _u16(x, npx * 16, "x"), _f32(t, npx * 2, "t"), _f32(tnorm, batch, "tnorm"),
                               border, batch, height, width, _ptr(ws), ws.numel(), C.byref(loss),
                               g.ctypes.data_as(C.POINTER(C.c_float)) if g is not None else None), "ac_cnn_grad")
    return loss.value, g


def ac_cnn_grad_residual(cnn: Cnn, x: torch.Tensor, rhat: torch.Tensor, kappa: torch.Tensor, lam: torch.Tensor,
                         rnorm: torch.Tensor, border: int, batch: int, height: int, width: int, ws: torch.Tensor,
                         want_grad: bool = False):
    """Residual-space loss (rhat [B,H,W,2], kappa [B,H,W], lam [B,2], rnorm [B], float32)."""
    import numpy as np
    npx = batch * height * width
    loss = C.c_double()
    g = np.zeros(L.load().ac_cnn_param_count(), dtype=np.float32) if want_grad else None
    check(L.load().ac_cnn_grad_residual(
        cnn.h, _u16(x, npx * 16, "x"), _f32(rhat, npx * 2, "rhat"), _f32(kappa, npx, "kappa"),
        _f32(lam, batch * 2, "lam"), _f32(rnorm, batch, "rnorm"), border, batch, height, width, _ptr(ws), ws.numel(),
        C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float)) if g is not None else None), "ac_cnn_grad_residual")
    return loss.value, g


def ac_cnn_adam_step(cnn: Cnn, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    check(L.load().ac_cnn_adam_step(cnn.h, lr, beta1, beta2, eps), "ac_cnn_adam_step")


def ac_cnn_make_inputs(p: Problem, cnn: Cnn, precision: int, rhat: torch.Tensor, x: torch.Tensor,
                       rscaled: torch.Tensor | None = None):
    """Network inputs x (bf16 bits) and, optionally, rhat_m / s_m in float32 (rscaled,
    [l_s][N][2]); returns the RMS scales s_m in slot order."""
    import numpy as np
    sc = np.empty(p.ns, dtype=np.float64)
    rs = None if rscaled is None else _f32(rscaled, p.ns * p.n * 2, "rscaled")
    check(L.load().ac_cnn_make_inputs(p.h, cnn.h, precision, _ptr(rhat), _u16(x, p.ns * p.n * 16, "x"),
                                      sc.ctypes.data_as(C.POINTER(C.c_double)), rs), "ac_cnn_make_inputs")
    return sc


def ac_ctx_set_graphs(ctx: Ctx, on: bool) -> None:
    check(L.load().ac_ctx_set_graphs(ctx.h, 1 if on else 0), "ac_ctx_set_graphs")


def ac_problem_create_multigrid(p: Problem) -> None:
    """Build the multigrid hierarchy of A used by AC_INNER_SP (owned by the problem)."""
    check(L.load().ac_problem_create_multigrid(p.h), "ac_problem_create_multigrid")


def ac_mg_workspace_size(p: Problem, nvec: int) -> int:
    n = C.c_size_t()
    check(L.load().ac_mg_workspace_size(p.h, nvec, C.byref(n)), "ac_mg_workspace_size")
    return n.value


def ac_mg_vcycle(p: Problem, shifts, b: torch.Tensor, u: torch.Tensor, ws: torch.Tensor) -> None:
    """u_q = V-cycle for (A - shifts[q] I) from b_q; b, u: len(shifts) * N float64."""
    nv = len(shifts)
    arr = (C.c_double * nv)(*[float(c) for c in shifts])
    check(L.load().ac_mg_vcycle(p.h, nv, arr, _f64(b, nv * p.n, "b"), _f64(u, nv * p.n, "u"), _ptr(ws),
                                ws.numel()), "ac_mg_vcycle")


def ac_problem_attach_cnn(p: Problem, cnn: Cnn | None) -> None:
    check(L.load().ac_problem_attach_cnn(p.h, cnn.h if cnn is not None else None), "ac_problem_attach_cnn")
    p._cnn = cnn  # keep the network alive while attached


def slot_order(p: Problem) -> list[int]:
    """Frequency m of each shift slot (real shifts first, then complex m = 1, 2, ...)."""
    real = [0] + ([p.ell // 2] if p.ell % 2 == 0 else [])
    return real + [m for m in range(1, (p.ell + 1) // 2)]


def ac_shifted_residual(p: Problem, precision: int, rhat: torch.Tensor, yhat: torch.Tensor):
    import numpy as np
    rel = np.empty(p.ns, dtype=np.float64)
    check(L.load().ac_shifted_residual(p.h, precision, _ptr(rhat), _ptr(yhat),
                                       rel.ctypes.data_as(C.POINTER(C.c_double))), "ac_shifted_residual")
    return rel


def ac_cnn_guess_workspace_size(p: Problem) -> int:
    n = C.c_size_t()
    check(L.load().ac_cnn_guess_workspace_size(p.h, C.byref(n)), "ac_cnn_guess_workspace_size")
    return n.value


def ac_cnn_guess(p: Problem, precision: int, rhat: torch.Tensor, x0hat: torch.Tensor, ws: torch.Tensor) -> int:
    """Writes the warm start's guesses into x0hat; returns the number of rejected slots."""
    rej = C.c_int()
    check(L.load().ac_cnn_guess(p.h, precision, _ptr(rhat), _ptr(x0hat), _ptr(ws), ws.numel(), C.byref(rej)),
          "ac_cnn_guess")
    return rej.value


def ac_cnn_set_inference(cnn: Cnn, fused: bool) -> None:
    check(L.load().ac_cnn_set_inference(cnn.h, 1 if fused else 0), "ac_cnn_set_inference")


def ac_cnn_set_guess_policy(cnn: Cnn, scaling: bool, accept_ratio: float = 1.0) -> None:
    check(L.load().ac_cnn_set_guess_policy(cnn.h, 1 if scaling else 0, accept_ratio), "ac_cnn_set_guess_policy")
