"""Pins of the oracle's spatial and all-at-once operators (not GPU).

Each check compares the oracle against something other than itself: an
independent textbook construction, a closed form of Appendix A, a dense
eigensolver, or a direct solve of the sequential chain of Section 1.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle.alloc import paper_operator_kappa
from synth import lognormal_kappa, random_block_vector, first_block_rhs


def _tridiag(n, periodic=False):
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    if periodic:
        T[0, n - 1] -= 1
        T[n - 1, 0] -= 1
    return T.tocsr()


@pytest.mark.parametrize("dim,nx,ny", [(1, 9, 1), (2, 7, 5)])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_constant_kappa_is_identity_plus_scaled_laplacian(dim, nx, ny, bc):
    """Constant kappa must give I + kappa(-Delta_h) built as a Kronecker sum of 1D
    second-difference matrices (the paper's operator of Section 5)."""
    kap = 3.7
    per = bc == "periodic"
    if dim == 1:
        L = _tridiag(nx, per)
    else:
        L = sp.kron(sp.identity(ny), _tridiag(nx, per)) + sp.kron(_tridiag(ny, per), sp.identity(nx))
    ref = sp.identity(nx * ny) + kap * L
    A = ops.build_A(dim, nx, ny, kap, bc)
    assert abs(A - ref).max() < 1e-13


def test_dirichlet_spectrum_appendix_a():
    nx, ny, kap = 8, 6, 12.5
    A = ops.build_A(2, nx, ny, kap).toarray()
    ev = np.linalg.eigvalsh(A)
    ref = np.sort(ops.dirichlet_eigs(2, nx, ny, kap).ravel())
    assert np.max(np.abs(ev - ref)) < 1e-11 * ref.max()


def test_sine_eigenvectors_appendix_a():
    n, kap = 11, 4.0
    A = ops.build_A(1, n, 1, kap)
    mu = ops.dirichlet_eigs_1d(n, kap)
    for j in range(1, n + 1):
        v = ops.sine_vector(n, j)
        assert abs(np.linalg.norm(v) - 1) < 1e-13
        assert np.linalg.norm(A @ v - mu[j - 1] * v) < 1e-12 * mu[j - 1]
    # 2D eigenvectors are tensor products V_i (x) V_j
    A2 = ops.build_A(2, n, n, kap)
    mu2 = ops.dirichlet_eigs(2, n, n, kap)
    v = np.kron(ops.sine_vector(n, 3), ops.sine_vector(n, 7))
    assert np.linalg.norm(A2 @ v - mu2[2, 6] * v) < 1e-12 * mu2.max()


def test_periodic_spectrum():
    nx, ny, kap = 6, 5, 2.0
    A = ops.build_A(2, nx, ny, kap, "periodic").toarray()
    ev = np.linalg.eigvalsh(A)
    assert np.max(np.abs(ev - np.sort(ops.periodic_eigs(2, nx, ny, kap).ravel()))) < 1e-12


def test_paper_operator_statements():
    """Appendix A: mu_min > 1; for large n_x mu_max ~ 1 + 8 nu/h^2 and mu_min ~ 1 + 2 nu pi^2."""
    ell = 10
    for nx in (50, 100, 500):
        kap = paper_operator_kappa(nx, ell)
        lo, hi = ops.constant_interval(2, nx, nx, kap)
        nu = 0.04 / (2 * ell - 4)
        assert lo > 1.0
        assert abs(hi - (1 + 8 * kap)) / hi < 2e-3 * (100 / nx) ** 2 + 1e-12
        assert abs(lo - (1 + 2 * nu * np.pi ** 2)) < 1e-2
    # n_x = 100, l = 10: nu/h^2 = 0.04/16 * 101^2
    assert abs(paper_operator_kappa(100, 10) - 25.5025) < 1e-12


@pytest.mark.parametrize("dim,nx,ny", [(1, 40, 1), (2, 12, 9)])
def test_variable_interval_encloses_spectrum(dim, nx, ny):
    kap = lognormal_kappa(nx, ny, 5.0, 3.0, 1.0, seed=3)
    lo, hi = ops.spectral_interval(dim, nx, ny, kap)
    ev = np.linalg.eigvalsh(ops.build_A(dim, nx, ny, kap).toarray())
    assert lo <= ev.min() + 1e-12 and ev.max() <= hi + 1e-9
    assert lo >= 1.0


def test_apply_calA_matches_explicit_matrix():
    nx, ny, ell = 6, 5, 4
    kap = lognormal_kappa(nx, ny, 2.0, 2.0, 0.7, seed=1)
    A = ops.build_A(2, nx, ny, kap)
    x = random_block_vector(nx * ny, ell, seed=5)
    calA = ops.build_calA(A, ell)
    assert np.linalg.norm(calA @ x - ops.apply_calA(A, x, ell)) < 1e-13 * np.linalg.norm(calA @ x)
    # explicit block structure of eq. (1)
    D = calA.toarray()
    n = nx * ny
    assert np.allclose(D[n:2 * n, 0:n], -np.eye(n))
    assert np.allclose(D[0:n, n:2 * n], 0.0)
    assert np.allclose(D[2 * n:3 * n, 2 * n:3 * n], A.toarray())


@pytest.mark.parametrize("ell", [2, 4, 7])
def test_all_at_once_equals_sequential(ell):
    """Section 1: solving the all-at-once system is the chain A x_1 = b_1, A x_{k+1} = x_k."""
    nx, ny = 9, 7
    kap = lognormal_kappa(nx, ny, 3.0, 2.0, 1.0, seed=2)
    A = ops.build_A(2, nx, ny, kap)
    b = first_block_rhs(nx * ny, ell, seed=0)
    x_seq = ops.sequential_solve(A, b, ell)
    x_dir = spla.spsolve(ops.build_calA(A, ell).tocsc(), b)
    assert np.linalg.norm(x_seq - x_dir) < 1e-13 * np.linalg.norm(x_dir)
    # the chain by hand for the first two blocks
    n = nx * ny
    x1 = np.linalg.solve(A.toarray(), b[:n])
    x2 = np.linalg.solve(A.toarray(), x1)
    assert np.allclose(x_seq[:n], x1, rtol=1e-13, atol=1e-15)
    assert np.allclose(x_seq[n:2 * n], x2, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("dim,nx,ny,ell,kappa", [(1, 31, 1, 4, 25.0), (2, 9, 7, 5, 3.0), (2, 16, 11, 10, 50.0)])
def test_closed_form_chain_equals_direct_solves(dim, nx, ny, ell, kappa):
    """Constant kappa, Dirichlet: the sine-transform chain equals the sparse LU chain and
    the direct solve of the assembled all-at-once matrix of eq. (1), for a rhs with every
    block nonzero (so the x_{k-1} coupling of every link is exercised)."""
    n = nx * (ny if dim == 2 else 1)
    b = random_block_vector(n, ell, seed=11)
    A = ops.build_A(dim, nx, ny, kappa)
    x_cf = ops.sequential_solve_closed_form(dim, nx, ny, kappa, b, ell)
    x_seq = ops.sequential_solve(A, b, ell)
    x_dir = spla.spsolve(ops.build_calA(A, ell).tocsc(), b)
    assert np.linalg.norm(x_cf - x_seq) < 1e-13 * np.linalg.norm(x_seq)
    assert np.linalg.norm(x_cf - x_dir) < 1e-13 * np.linalg.norm(x_dir)


def test_closed_form_chain_single_mode():
    """One sine eigenvector as b_1 (Appendix A): x_k = mu^{-k} V_j exactly."""
    nx, ell, kappa, j = 20, 6, 7.0, 3
    v = ops.sine_vector(nx, j)
    mu = 1.0 + 4.0 * kappa * np.sin(j * np.pi / (2 * (nx + 1))) ** 2
    b = np.zeros(ell * nx)
    b[:nx] = v
    x = ops.sequential_solve_closed_form(1, nx, 1, kappa, b, ell).reshape(ell, nx)
    for k in range(ell):
        assert np.allclose(x[k], v / mu ** (k + 1), rtol=1e-13, atol=1e-16)


def test_varying_blocks_reduce_to_constant_blocks():
    rng = np.random.default_rng(21)
    nx, ny, ell = 6, 5, 4
    kap = rng.uniform(0.5, 3.0, nx * ny)
    A = ops.build_A(2, nx, ny, kap)
    x = rng.standard_normal(ell * nx * ny)
    assert np.allclose(ops.apply_calA_blocks([A] * ell, x), ops.apply_calA(A, x, ell), rtol=0, atol=1e-14)
    assert abs(ops.build_calA_blocks([A] * ell) - ops.build_calA(A, ell)).max() == 0


def test_varying_blocks_sequential_equals_direct_solve():
    rng = np.random.default_rng(22)
    nx, ny, ell = 5, 4, 5
    kaps = rng.uniform(0.2, 4.0, (ell, nx * ny))
    As = [ops.build_A(2, nx, ny, k) for k in kaps]
    b = rng.standard_normal(ell * nx * ny)
    M = ops.build_calA_blocks(As).toarray()
    # block structure by hand: A_k on the diagonal, -I below it
    n = nx * ny
    for k in range(ell):
        assert np.array_equal(M[k * n:(k + 1) * n, k * n:(k + 1) * n], As[k].toarray())
        if k > 0:
            assert np.array_equal(M[k * n:(k + 1) * n, (k - 1) * n:k * n], -np.eye(n))
    x = ops.sequential_solve_blocks(As, b)
    assert np.linalg.norm(M @ x - b) < 1e-12 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.solve(M, b), rtol=0, atol=1e-12)


def test_mean_kappa_gives_the_mean_block():
    """A is affine in the cell coefficients: A(mean kappa_k) = mean A(kappa_k)."""
    rng = np.random.default_rng(23)
    nx, ny, ell = 7, 3, 6
    kaps = rng.uniform(0.1, 5.0, (ell, nx * ny))
    Am = ops.build_A(2, nx, ny, ops.mean_block_kappa(kaps))
    mean = sum(ops.build_A(2, nx, ny, k) for k in kaps) / ell
    assert abs(Am - mean).max() < 1e-13
