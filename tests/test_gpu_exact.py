"""Exact P_alpha^{-1} on the GPU for a constant coefficient (AC_INNER_EXACT): the time-DFT
of Section 2.2, direct shifted solves (A - lambda_m I) through the sine transform of
Appendix A along x and tridiagonal elimination along y, and the inverse time-DFT.

Parity: element-wise against the oracle's apply_prec_exact (sparse LU solves of eq. (4))
on small ragged grids; at full size (2048^2, l = 10) the property P_alpha z = r, with
P_alpha = I (x) A - C_alpha (x) I of eq. (2), evaluated by the library's calA product plus
the alpha z_l corner term.  Outer solves: FGMRES and the outer Chebyshev iteration reach
the oracle's iteration counts with the same preconditioner."""

import numpy as np
import pytest
import torch

from oracle import operators as ops
from oracle import precond as pc
from oracle.bounds import cor1_interval
from oracle.krylov import fgmres, outer_chebyshev
from paper_2506_03947_amd import api
from synth import first_block_rhs, lognormal_kappa, random_block_vector
from tests import gpu_util as G

L = api.L
pytestmark = pytest.mark.gpu


def f32_tol(nx, ell, alpha):
    """float32 inner arithmetic: each sine transform is a length-n_x sum (error growing like
    sqrt(n_x) ulps), the tridiagonal elimination is contracting, and the inverse time
    transform scales block k by alpha^{-k/l} <= alpha^{-(l-1)/l}."""
    return 16.0 * np.sqrt(nx) * alpha ** (-(ell - 1) / ell) * 2.0 ** -24


def _exact(p, precision, r):
    opts = api.Opts(precision=precision, inner=L.AC_INNER_EXACT)
    z = torch.empty_like(r)
    api.ac_apply_prec(p, opts, r, z, api.workspace(api.ac_prec_workspace_size(p, opts)))
    return G.host(z)


@pytest.mark.parametrize("dim,nx,ny,ell,alpha,kappa", [
    (2, 23, 17, 4, 1e-2, 3.7),
    (2, 31, 9, 5, 1.0, 0.8),
    (2, 1, 13, 6, 1e-2, 2.0),
    (2, 40, 1, 3, 0.5, 5.0),
    (1, 57, 1, 7, 1e-2, 11.0),
    (2, 70, 66, 10, 1e-2, 25.0),
    (2, 17, 15, 2, 0.3, 4.0),      # only real shifts
    (2, 12, 19, 3, 1e-2, 6.0),     # one real, one complex shift
    (2, 20, 18, 16, 1e-3, 9.0),    # the largest l
    (1, 1, 1, 4, 0.5, 2.0),        # a single point
])
def test_exact_prec_matches_oracle(dim, nx, ny, ell, alpha, kappa):
    A = ops.build_A(dim, nx, ny, kappa)
    n = nx * ny
    r = random_block_vector(n, ell, seed=nx + ell)
    ref = pc.apply_prec_exact(A, r, ell, alpha)
    p = G.problem(dim, nx, ny, kappa, ell, alpha)
    z64 = _exact(p, L.AC_PREC_FP64, G.dev(r))
    assert G.rel(z64, ref) < 1e-12, G.rel(z64, ref)
    for prec in (L.AC_PREC_MIXED_FP32K, L.AC_PREC_MIXED_BF16K):
        z32 = _exact(p, prec, G.dev(r))
        assert G.rel(z32, ref) < f32_tol(nx, ell, alpha), (prec, G.rel(z32, ref))


def _palpha(p, z, ell, n, alpha):
    """P_alpha z = calA z - alpha (e_1 e_l^T (x) I) z (eq. (2)), on the device."""
    y = torch.empty_like(z)
    api.ac_apply_A(p, z, y)
    y[:n] -= alpha * z[(ell - 1) * n:]
    return y


def test_exact_prec_full_size_property():
    """2048^2, l = 10: P_alpha z = r for the float64 path; the float32 path against it."""
    nx = ny = 2048
    ell, alpha, kappa = 10, 1e-2, 40.0
    n = nx * ny
    p = G.problem(2, nx, ny, kappa, ell, alpha)
    g = torch.Generator(device="cuda:0").manual_seed(7)
    r = torch.randn(ell * n, dtype=torch.float64, device="cuda:0", generator=g)
    zs = {}
    for prec in (L.AC_PREC_FP64, L.AC_PREC_MIXED_FP32K):
        opts = api.Opts(precision=prec, inner=L.AC_INNER_EXACT)
        zs[prec] = torch.empty_like(r)
        api.ac_apply_prec(p, opts, r, zs[prec], api.workspace(api.ac_prec_workspace_size(p, opts)))
    z = zs[L.AC_PREC_FP64]
    res = float(torch.linalg.vector_norm(_palpha(p, z, ell, n, alpha) - r) / torch.linalg.vector_norm(r))
    d32 = float(torch.linalg.vector_norm(zs[L.AC_PREC_MIXED_FP32K] - z) / torch.linalg.vector_norm(z))
    print(f"exact P_alpha at 2048^2, l=10: |P z - r|/|r| = {res:.3e}, float32 vs float64 {d32:.3e}", flush=True)
    assert res < 1e-11
    assert d32 < f32_tol(nx, ell, alpha)


def test_exact_prec_full_size_closed_form():
    """2048^2 at l = 2 against the oracle's closed form (orthonormal DST-I of the whole
    grid, Appendix A), element by element."""
    nx = ny = 2048
    ell, alpha, kappa = 2, 0.3, 7.0
    n = nx * ny
    r = random_block_vector(n, ell, seed=5)
    ref = pc.apply_prec_closed_form(2, nx, ny, kappa, r, ell, alpha)
    p = G.problem(2, nx, ny, kappa, ell, alpha)
    z = _exact(p, L.AC_PREC_FP64, G.dev(r))
    assert G.rel(z, ref) < 1e-12, G.rel(z, ref)


@pytest.mark.parametrize("alpha", [1e-2, 1.0])
def test_exact_fgmres_matches_oracle_counts(alpha):
    nx, ell, kappa = 48, 10, 30.0
    A = ops.build_A(2, nx, nx, kappa)
    b = first_block_rhs(nx * nx, ell, seed=4)
    _, ref = fgmres(lambda v: ops.apply_calA(A, v, ell), b, lambda v: pc.apply_prec_exact(A, v, ell, alpha),
                    tol=1e-10, m=30)
    p = G.problem(2, nx, nx, kappa, ell, alpha)
    opts = api.Opts(precision=L.AC_PREC_FP64, inner=L.AC_INNER_EXACT, tol=1e-10, restart_m=30, max_outer=100)
    x = G.dev(np.zeros_like(b))
    info = api.ac_solve(p, opts, G.dev(b), x, api.workspace(api.ac_solve_workspace_size(p, opts)))
    assert info["converged"] and info["rel_residual_true"] < 1e-10
    assert abs(info["outer_iters"] - ref["iterations"]) <= 1, (info["outer_iters"], ref["iterations"])
    # no inner products with A: l per calA only
    assert info["matvecs_A"] == info["outer_iters"] * ell + info["restarts"] * ell + ell
    assert G.rel(G.host(x), ops.sequential_solve(A, b, ell)) < 1e-8


def test_exact_outer_chebyshev_matches_oracle():
    nx, ell, alpha, kappa = 40, 10, 1e-2, 30.0
    A = ops.build_A(2, nx, nx, kappa)
    lo, hi = ops.constant_interval(2, nx, nx, kappa)
    b = first_block_rhs(nx * nx, ell, seed=2)
    a, bnd = cor1_interval(lo, ell, alpha)
    x_ref, it_ref = outer_chebyshev(lambda v: ops.apply_calA(A, v, ell), b,
                                    lambda v: pc.apply_prec_exact(A, v, ell, alpha), a, bnd, 1e-6)
    p = G.problem(2, nx, nx, kappa, ell, alpha, bounds=(lo, hi))
    opts = api.Opts(precision=L.AC_PREC_FP64, inner=L.AC_INNER_EXACT, tol=1e-6, restart_m=1, max_outer=100,
                    outer=L.AC_OUTER_CHEBYSHEV)
    x = G.dev(np.zeros_like(b))
    info = api.ac_solve(p, opts, G.dev(b), x, api.workspace(api.ac_solve_workspace_size(p, opts)))
    assert info["converged"] and abs(info["outer_iters"] - it_ref) <= 1, (info["outer_iters"], it_ref)
    assert G.rel(G.host(x), x_ref) < (1e-9 if info["outer_iters"] == it_ref else 1e-5)


def test_exact_varying_blocks_with_constant_mean():
    """Varying diagonal blocks whose pointwise mean is constant: the exact preconditioner
    is P_alpha(A_hat) with A_hat = A(mean kappa) (representative block)."""
    nx, ell, alpha = 24, 4, 1e-2
    levels = np.array([2.0, 3.0, 5.0, 6.0])
    kb = np.repeat(levels[:, None], nx * nx, axis=1).reshape(-1)
    Ahat = ops.build_A(2, nx, nx, float(levels.mean()))
    r = random_block_vector(nx * nx, ell, seed=9)
    ref = pc.apply_prec_exact(Ahat, r, ell, alpha)
    p = api.ac_problem_create_blocks(G.ctx(), 2, nx, nx, G.dev(kb), ell, alpha)
    z = _exact(p, L.AC_PREC_FP64, G.dev(r))
    assert G.rel(z, ref) < 1e-12


def test_exact_rejects_unsupported():
    nx, ell = 32, 4
    opts = api.Opts(precision=L.AC_PREC_FP64, inner=L.AC_INNER_EXACT)
    r = torch.zeros(ell * nx * nx, dtype=torch.float64, device="cuda:0")
    z = torch.empty_like(r)
    ws = api.workspace(1 << 26)
    kap = lognormal_kappa(nx, nx, 5.0, 6.0, 0.5, seed=1)
    for p in (G.problem(2, nx, nx, kap, ell, 1e-2),
              G.problem(2, nx, nx, 2.0, ell, 1e-2, bc=L.AC_BC_PERIODIC)):
        with pytest.raises(L.AlphacircError) as e:
            api.ac_apply_prec(p, opts, r, z, ws)
        assert e.value.status == L.AC_ERR_UNSUPPORTED
    p = G.problem(2, nx, nx, 2.0, ell, 1e-2)
    with pytest.raises(L.AlphacircError) as e:
        api.ac_shifted_cheb(p, opts, torch.zeros(1 << 16, device="cuda:0"), None,
                            torch.zeros(1 << 16, device="cuda:0"), ws)
    assert e.value.status == L.AC_ERR_UNSUPPORTED
