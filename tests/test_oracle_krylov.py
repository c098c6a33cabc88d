"""Pins of the oracle's outer solvers (not GPU).

* FGMRES / right-preconditioned GMRES solutions against the sequential direct
  solve of Section 1 (the all-at-once solution is unique, so any converged
  Krylov iterate must approach it within cond * tolerance);
* the paper's outer Chebyshev semi-iteration with Corollary 1 bounds against the
  NC2 / NC1 iteration counts of Table 3 (alpha = 0.01, eta = 0.2).  The paper's
  own duplicate point (n_x = 100, l = 10 appears in Tables 3 and 4) differs by
  one iteration, so counts are pinned to +-1 (NC2) and +-2 (NC1).
"""

import numpy as np
import pytest

from oracle import operators as ops
from oracle import precond as pc
from oracle.alloc import alg1_allocation, nc1_allocation, paper_operator_kappa
from oracle.bounds import cor1_interval
from oracle.krylov import fgmres, outer_chebyshev
from synth import first_block_rhs, lognormal_kappa


def _problem(nx=16, ny=12, ell=4, seed=0):
    kap = lognormal_kappa(nx, ny, 5.0, 3.0, 1.0, seed=seed)
    A = ops.build_A(2, nx, ny, kap)
    lo, hi = ops.spectral_interval(2, nx, ny, kap)
    b = first_block_rhs(nx * ny, ell, seed=0)
    return A, kap, lo, hi, b


def test_unpreconditioned_gmres_matches_sequential():
    A, kap, lo, hi, b = _problem()
    ell = 4
    x_seq = ops.sequential_solve(A, b, ell)
    x, info = fgmres(lambda v: ops.apply_calA(A, v, ell), b, None, tol=1e-12, m=30, max_outer=3000)
    assert info["rel_residual"] <= 1e-12
    assert np.linalg.norm(x - x_seq) / np.linalg.norm(x_seq) < 1e-9


@pytest.mark.parametrize("alpha", [1e-1, 1e-2, 1e-3])
def test_exact_preconditioner_few_iterations(alpha):
    A, kap, lo, hi, b = _problem()
    ell = 4
    x_seq = ops.sequential_solve(A, b, ell)
    x, info = fgmres(lambda v: ops.apply_calA(A, v, ell), b,
                     lambda r: pc.apply_prec_exact(A, r, ell, alpha), tol=1e-12, m=30)
    assert info["rel_residual"] <= 1e-12
    # Corollary 1: eigenvalues in [1, 1 + alpha/(mu^l - alpha)] -> very few iterations
    assert info["iterations"] <= 8
    assert np.linalg.norm(x - x_seq) / np.linalg.norm(x_seq) < 1e-10


def test_nested_chebyshev_fgmres_matches_sequential():
    A, kap, lo, hi, b = _problem(ell=6)
    ell, alpha = 6, 1e-2
    x_seq = ops.sequential_solve(A, b, ell)
    x, info = fgmres(lambda v: ops.apply_calA(A, v, ell), b,
                     lambda r: pc.apply_prec_nc(A, r, ell, alpha, lo, hi, 10), tol=1e-12, m=20)
    assert info["rel_residual"] <= 1e-12
    assert np.linalg.norm(x - x_seq) / np.linalg.norm(x_seq) < 1e-10
    x0, info0 = fgmres(lambda v: ops.apply_calA(A, v, ell), b, None, tol=1e-12, m=20, max_outer=5000)
    assert info["iterations"] < info0["iterations"]


def test_fgmres_restart_path():
    A, kap, lo, hi, b = _problem(ell=4)
    ell = 4
    x_seq = ops.sequential_solve(A, b, ell)
    x, info = fgmres(lambda v: ops.apply_calA(A, v, ell), b,
                     lambda r: pc.apply_prec_nc(A, r, ell, 1e-2, lo, hi, 3), tol=1e-11, m=4, max_outer=500)
    assert info["restarts"] > 1
    assert info["rel_residual"] <= 1e-11
    assert np.linalg.norm(x - x_seq) / np.linalg.norm(x_seq) < 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("nx,method,expected,slack", [(50, "NC2", 10, 1), (50, "NC1", 13, 2),
                                                      (100, "NC2", 8, 1), (100, "NC1", 12, 2)])
def test_outer_chebyshev_table3(nx, method, expected, slack):
    ell, alpha, eta = 10, 0.01, 0.2
    kap = paper_operator_kappa(nx, ell)
    lo, hi = ops.constant_interval(2, nx, nx, kap)
    A = ops.build_A(2, nx, nx, kap)
    budget = ell * nx * eta
    p = alg1_allocation(ell, budget, lo, hi, alpha) if method == "NC2" else nc1_allocation(ell, budget)
    a, bnd = cor1_interval(lo, ell, alpha)
    b = first_block_rhs(nx * nx, ell, seed=0)
    x, it = outer_chebyshev(lambda v: ops.apply_calA(A, v, ell), b,
                            lambda r: pc.apply_prec_nc(A, r, ell, alpha, lo, hi, p), a, bnd, 1e-6)
    assert abs(it - expected) <= slack, it
    r = b - ops.apply_calA(A, x, ell)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-6
