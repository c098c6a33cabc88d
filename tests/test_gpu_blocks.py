"""Varying diagonal blocks A_1..A_l (Conclusions): calA against the oracle, P^{-1}
through the representative block A(mean kappa) against the oracle's nested
Chebyshev on that block, and FGMRES solves against the sequential chain of solves."""

import numpy as np
import pytest

from oracle import operators as ops
from oracle import precond as pc
from paper_2506_03947_amd import api
from synth import first_block_rhs, lognormal_kappa
from tests import gpu_util as G

L = api.L
pytestmark = pytest.mark.gpu


def _blocks(nx, ny, ell, seed, drift=1.0):
    """kappa_k = kappa0 exp(g + drift * (k / l) h): a log-normal field whose pattern
    drifts through the window (g, h independent fields)."""
    g = np.log(lognormal_kappa(nx, ny, 1.0, 6.0, 1.0, seed=seed))
    h = np.log(lognormal_kappa(nx, ny, 1.0, 6.0, 1.0, seed=seed + 1))
    return np.stack([20.0 * np.exp(g + drift * (k / ell) * h) for k in range(ell)])


@pytest.mark.parametrize("nx,ny,ell", [(96, 64, 4), (131, 70, 7), (256, 128, 10)])
def test_apply_A_varying_blocks(nx, ny, ell):
    kaps = _blocks(nx, ny, ell, 3)
    p = api.ac_problem_create_blocks(G.ctx(), 2, nx, ny, G.dev(kaps.reshape(-1)), ell, 1e-2)
    As = [ops.build_A(2, nx, ny, k) for k in kaps]
    x = np.random.default_rng(ell).standard_normal(ell * nx * ny)
    y = G.dev(np.zeros_like(x))
    api.ac_apply_A(p, G.dev(x), y)
    assert G.rel(G.host(y), ops.apply_calA_blocks(As, x)) < 1e-14
    # the preconditioner is that of the mean block
    lo, hi = api.ac_spectral_bounds(p)
    A_hat = ops.build_A(2, nx, ny, ops.mean_block_kappa(kaps))
    opts = api.Opts(precision=L.AC_PREC_FP64, p=6)
    z = G.dev(np.zeros_like(x))
    api.ac_apply_prec(p, opts, G.dev(x), z, api.workspace(api.ac_prec_workspace_size(p, opts)))
    assert G.rel(G.host(z), pc.apply_prec_nc(A_hat, x, ell, 1e-2, lo, hi, 6)) < 1e-12


@pytest.mark.parametrize("precision", [L.AC_PREC_FP64, L.AC_PREC_MIXED_BF16K])
def test_solve_varying_blocks(precision):
    """The further the blocks drift from their mean, the more outer iterations the
    representative-block preconditioner needs (oracle, 64 x 48, l = 8, p = 10: 151
    iterations for equal blocks, 195 / 234 / 389 for drift 0.5 / 1 / 1.5)."""
    nx, ny, ell = 96, 64, 8
    kaps = _blocks(nx, ny, ell, 5, drift=0.5)
    p = api.ac_problem_create_blocks(G.ctx(), 2, nx, ny, G.dev(kaps.reshape(-1)), ell, 1e-2)
    As = [ops.build_A(2, nx, ny, k) for k in kaps]
    b = first_block_rhs(nx * ny, ell, seed=2)
    opts = api.Opts(precision=precision, p=10, tol=1e-10, restart_m=16, max_outer=2000)
    x = G.dev(np.zeros_like(b))
    info = api.ac_solve(p, opts, G.dev(b), x, api.workspace(api.ac_solve_workspace_size(p, opts)))
    assert info["converged"] and info["rel_residual_true"] <= 1e-10, info
    ref = ops.sequential_solve_blocks(As, b)
    assert G.rel(G.host(x), ref) < 1e-7
    if precision == L.AC_PREC_FP64:
        # the oracle's FGMRES with the same preconditioner takes about as many steps
        from oracle.krylov import fgmres
        lo, hi = api.ac_spectral_bounds(p)
        A_hat = ops.build_A(2, nx, ny, ops.mean_block_kappa(kaps))
        _, oinfo = fgmres(lambda v: ops.apply_calA_blocks(As, v), b,
                          lambda v: pc.apply_prec_nc(A_hat, v, ell, 1e-2, lo, hi, 10), tol=1e-10, m=16,
                          max_outer=2000)
        assert abs(info["outer_iters"] - oinfo["iterations"]) <= 0.05 * oinfo["iterations"] + 3, (info, oinfo)
    # the outer residual is the varying-block one: recompute it on the host
    r = b - ops.apply_calA_blocks(As, G.host(x))
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_varying_blocks_errors():
    nx, ny, ell = 32, 32, 4
    kaps = _blocks(nx, ny, ell, 7)
    bad = kaps.copy()
    bad[2, 5] = -1.0
    with pytest.raises(api.L.AlphacircError):
        api.ac_problem_create_blocks(G.ctx(), 2, nx, ny, G.dev(bad.reshape(-1)), ell, 1e-2)
    p = api.ac_problem_create_blocks(G.ctx(), 2, nx, ny, G.dev(kaps.reshape(-1)), ell, 1e-2)
    opts = api.Opts(p=4, outer=L.AC_OUTER_CHEBYSHEV, restart_m=1, tol=1e-6)
    b = G.dev(np.ones(ell * nx * ny))
    with pytest.raises(api.L.AlphacircError):
        api.ac_solve(p, opts, b, G.dev(np.zeros(ell * nx * ny)), api.workspace(api.ac_solve_workspace_size(p, opts)))
    q = G.problem(2, nx, ny, 5.0, ell, 1e-2)
    bopts = api.Opts(p=4)
    with pytest.raises(api.L.AlphacircError):
        api.ac_batch_workspace_size(G.ctx(), [p, q], bopts)
