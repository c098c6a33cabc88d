"""CPU pins of the saddle-point preconditioner P_SP (Section 4) and of the multigrid
V-cycle that applies P_D (oracle/saddle.py, oracle/multigrid.py).

Paper pins: the saddle system of eq. (saddlesystem) reproduces the complex shifted solve;
Theorem 5's eigenvalue intervals for P_D^{-1} S; P_SP with many exact-P_D iterations is
P_alpha (eq. (4)).  Library pins: preconditioned MINRES and CG iterates equal scipy's
(the k-th iterate of each is unique); the multigrid (no paper definition, the paper uses
a black-box AMG) is pinned by properties: fine level = A, symmetric and positive
definite cycle, exact on a coarsest-only grid, linear interpolation reproduces linear
functions, and an h-independent contraction factor."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import multigrid as mg
from oracle import operators as ops
from oracle import precond as pc
from oracle import saddle as sd
from synth import lognormal_kappa, random_block_vector


def _lam(ell, alpha, m):
    return complex(pc.shifts(ell, alpha)[m])


@pytest.mark.parametrize("m", [1, 2, 4])
def test_saddle_system_is_the_complex_solve(m):
    nx, ny, ell, alpha = 9, 7, 6, 0.4
    A = ops.build_A(2, nx, ny, lognormal_kappa(nx, ny, 3.0, 3.0, 0.7, seed=1))
    lam = _lam(ell, alpha, m)
    rng = np.random.default_rng(m)
    b = rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)
    x = spla.spsolve((A - lam * sp.identity(nx * ny)).astype(complex).tocsc(), b)
    u = spla.spsolve(sd.saddle_matrix(A, lam).tocsc(), sd.saddle_rhs(b, lam))
    assert np.allclose(sd.saddle_solution(u, lam), x, rtol=1e-12, atol=1e-12)
    # the saddle matrix has the (Phi, Psi; Psi, -Phi) structure with Phi = |Im lambda| I
    S = sd.saddle_matrix(A, lam).toarray()
    n = nx * ny
    assert np.allclose(S[:n, :n], abs(lam.imag) * np.eye(n)) and np.allclose(S[n:, n:], -S[:n, :n])
    assert np.allclose(S[:n, n:], S[n:, :n]) and np.allclose(S[:n, n:], S[:n, n:].T)


@pytest.mark.parametrize("alpha,kappa", [(1.0, 5.0), (0.01, 40.0), (0.5, "lognormal")])
def test_theorem5_eigenvalues(alpha, kappa):
    nx, ny, ell = 8, 6, 10
    kap = lognormal_kappa(nx, ny, 10.0, 3.0, 1.0, seed=4) if kappa == "lognormal" else kappa
    A = ops.build_A(2, nx, ny, kap)
    n = nx * ny
    for m in range(1, ell):
        if 2 * m == ell:
            continue
        lam = _lam(ell, alpha, m)
        S = sd.saddle_matrix(A, lam).toarray()
        B = (A - sd.pd_shift(lam) * sp.identity(n)).toarray()
        P = np.block([[B, np.zeros_like(B)], [np.zeros_like(B), B]])
        ev = np.linalg.eigvals(np.linalg.solve(P, S))
        assert np.max(np.abs(ev.imag)) < 1e-10
        mag = np.abs(ev.real)
        assert mag.min() >= 1 / np.sqrt(2) - 1e-12 and mag.max() <= 1 + 1e-12
        # P_D is SPD (mu_min > Re lambda)
        assert np.linalg.eigvalsh(B).min() > 0


def test_minres_and_pcg_match_scipy():
    nx, ny = 10, 8
    A = ops.build_A(2, nx, ny, lognormal_kappa(nx, ny, 20.0, 3.0, 1.0, seed=2))
    n = nx * ny
    L = mg.hierarchy(2, nx, ny, lognormal_kappa(nx, ny, 20.0, 3.0, 1.0, seed=2))
    lam = _lam(8, 0.3, 3)
    S = sd.saddle_matrix(A, lam)
    c = sd.pd_shift(lam)
    Minv = lambda r: np.concatenate([mg.vcycle(L, r[:n], c), mg.vcycle(L, r[n:], c)])
    M = spla.LinearOperator((2 * n, 2 * n), matvec=Minv)
    b = np.random.default_rng(0).standard_normal(2 * n)
    for k in (1, 3, 7):
        ref, _ = spla.minres(S, b, M=M, maxiter=k, rtol=1e-300)
        got = sd.minres(lambda v: S @ v, b, Minv, k)
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref), k
    B = (A - 0.7 * sp.identity(n)).tocsr()
    Mr = spla.LinearOperator((n, n), matvec=lambda r: mg.vcycle(L, r, 0.7))
    br = b[:n]
    for k in (1, 4, 9):
        ref, _ = spla.cg(B, br, M=Mr, maxiter=k, rtol=1e-300)
        got = sd.pcg(lambda v: B @ v, br, lambda r: mg.vcycle(L, r, 0.7), k)
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref), k


def test_minres_residual_is_monotone_and_converges():
    nx, ny = 12, 12
    A = ops.build_A(2, nx, ny, 30.0)
    lam = _lam(10, 0.01, 2)
    S = sd.saddle_matrix(A, lam)
    c = sd.pd_shift(lam)
    n = nx * ny
    Pd = (A - c * sp.identity(n)).tocsc()
    Minv = lambda r: np.concatenate([spla.spsolve(Pd, r[:n]), spla.spsolve(Pd, r[n:])])
    b = np.random.default_rng(1).standard_normal(2 * n)
    Pfull = sp.bmat([[Pd, None], [None, Pd]]).tocsc()
    prev = np.inf
    for k in range(1, 16):
        x = sd.minres(lambda v: S @ v, b, Minv, k)
        r = b - S @ x
        res = np.sqrt(r @ spla.spsolve(Pfull, r))  # MINRES minimises the P_D^{-1} norm
        assert res <= prev * (1 + 1e-12)
        prev = res
    assert prev < 1e-8 * np.sqrt(b @ spla.spsolve(Pfull, b))


def test_multigrid_fine_level_and_coarsest():
    kap = lognormal_kappa(13, 11, 5.0, 3.0, 1.0, seed=3)
    L = mg.hierarchy(2, 13, 11, kap)
    A = ops.build_A(2, 13, 11, kap)
    assert abs(mg.level_matrix(L[0]) - A).max() < 1e-14 * abs(A).max()
    assert L[-1].nx * L[-1].ny <= 4
    L1 = mg.hierarchy(1, 2, 1, [3.0, 5.0])
    assert len(L1) == 1
    b = np.array([1.0, -2.0])
    x = mg.vcycle(L1, b, 0.4)
    assert np.allclose(mg.level_matrix(L1[0], 0.4) @ x, b, atol=1e-14)


@pytest.mark.parametrize("dim,nx,ny", [(2, 16, 12), (2, 13, 11), (1, 40, 1), (2, 1, 9), (2, 7, 2)])
def test_multigrid_cycle_symmetric_positive_definite(dim, nx, ny):
    n = nx * (ny if dim == 2 else 1)
    kap = lognormal_kappa(nx, max(ny, 1), 20.0, 3.0, 1.0, seed=nx)[:n]
    L = mg.hierarchy(dim, nx, ny, kap)
    B = np.column_stack([mg.vcycle(L, e, 0.6) for e in np.eye(n)])
    assert np.allclose(B, B.T, atol=1e-13 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_multigrid_interpolation_reproduces_linear():
    for n in (8, 9):
        f = mg.fine_level(1, n, 1, 1.0)
        c = mg.coarsen(f)
        P = mg.prolongation(f, c)
        xc = np.arange(c.nx) * 2 + 2.0     # coarse point J sits at fine position 2J + 2
        xf = np.arange(n) + 1.0            # fine point i at i + 1
        got = P @ xc
        # interior points (both coarse neighbours present) are exact; the zero boundary
        # value is linear interpolation towards 0 at position 0
        assert np.allclose(got[:2 * (c.nx - 1) + 2], xf[:2 * (c.nx - 1) + 2])


@pytest.mark.parametrize("nx,kappa", [(32, 100.0), (64, 100.0), (64, 1e4), (64, "lognormal"), (45, 300.0)])
def test_multigrid_contraction(nx, kappa):
    kap = lognormal_kappa(nx, nx, 50.0, 10.0, 1.0, seed=0) if kappa == "lognormal" else kappa
    L = mg.hierarchy(2, nx, nx, kap)
    A = mg.level_matrix(L[0], 0.6)
    e = np.random.default_rng(0).standard_normal(nx * nx)
    hist = []
    for _ in range(10):
        e = e - mg.vcycle(L, A @ e, 0.6)
        hist.append(np.linalg.norm(e))
    rate = (hist[-1] / hist[-4]) ** (1 / 3)
    assert rate < 0.3, rate


def test_apply_prec_sp_tends_to_exact():
    nx, ny, ell, alpha = 10, 9, 6, 0.05
    kap = lognormal_kappa(nx, ny, 10.0, 3.0, 0.8, seed=6)
    A = ops.build_A(2, nx, ny, kap)
    r = random_block_vector(nx * ny, ell, seed=1)
    ref = pc.apply_prec_exact(A, r, ell, alpha)
    L = mg.hierarchy(2, nx, ny, kap)
    errs = [np.linalg.norm(sd.apply_prec_sp(A, r, ell, alpha, k, L) - ref) / np.linalg.norm(ref) for k in (2, 6, 30)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-10, errs
    # with exact P_D, MINRES needs few steps (Theorem 5 clusters the spectrum in two intervals)
    e_ex = np.linalg.norm(sd.apply_prec_sp(A, r, ell, alpha, 12) - ref) / np.linalg.norm(ref)
    assert e_ex < 1e-6, e_ex


def test_apply_prec_sp_conjugate_branches_agree():
    """Slices m and l-m run the two sign branches of the saddle form; their solutions are
    complex conjugates (Hermitian symmetry of the transform)."""
    nx, ny, ell, alpha = 8, 7, 8, 0.2
    kap = lognormal_kappa(nx, ny, 5.0, 3.0, 0.5, seed=2)
    A = ops.build_A(2, nx, ny, kap)
    L = mg.hierarchy(2, nx, ny, kap)
    r = random_block_vector(nx * ny, ell, seed=3)
    y = sd.apply_prec_sp(A, r, ell, alpha, 5, L, return_complex=True)
    assert np.max(np.abs(y.imag)) < 1e-12 * np.max(np.abs(y.real))


@pytest.mark.parametrize("nx", [15, 16, 9])
def test_multigrid_coarse_faces_are_halved_schur_complement_1d(nx):
    """1D coarse-face rule against exact elimination: removing the fine points that are
    not coarse points (0, 2, 4, ...) from the pure-diffusion part A - I of the fine level
    leaves a tridiagonal Schur complement on the coarse points; its off-diagonals are the
    series conductances ab/(a + b) of the two fine faces between coarse neighbours, and
    its Dirichlet terms those of a fine interior face in series with the boundary face.
    The coarse level's faces (spacing 2h, full-weighting scale 1/2) are exactly half of
    it, on odd and even sizes (the even size's high end keeps its own boundary face)."""
    kap = np.exp(np.random.default_rng(nx).normal(0.0, 1.5, nx))
    fine = mg.fine_level(1, nx, 1, kap)
    coarse = mg.coarsen(fine)
    Ld = (mg.level_matrix(fine) - sp.identity(nx)).toarray()
    C = np.arange(1, nx, 2)
    F = np.setdiff1d(np.arange(nx), C)
    S = Ld[np.ix_(C, C)] - Ld[np.ix_(C, F)] @ np.linalg.solve(Ld[np.ix_(F, F)], Ld[np.ix_(F, C)])
    Lc = (mg.level_matrix(coarse) - sp.identity(len(C))).toarray()
    assert Lc.shape == S.shape
    assert np.allclose(Lc, 0.5 * S, rtol=1e-13, atol=1e-13)


def test_multigrid_constant_kappa_coarse_level_is_rediscretisation():
    """Constant kappa on a 15 x 15 grid: the coarse level is I + (kappa/4)(-Delta) on the
    7 x 7 coarse points, the textbook rediscretisation at twice the spacing (kappa =
    nu/h^2 becomes nu/(2h)^2)."""
    kappa = 12.0
    levels = mg.hierarchy(2, 15, 15, kappa)
    assert (levels[1].nx, levels[1].ny) == (7, 7)
    ref = ops.build_A(2, 7, 7, kappa / 4.0)
    assert np.allclose(mg.level_matrix(levels[1]).toarray(), ref.toarray(), rtol=1e-14, atol=1e-13)
