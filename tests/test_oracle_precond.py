"""Pins of the oracle's preconditioner (not GPU).

* eq. (2): dense brute-force P_alpha against the DFT route of eq. (4);
* eq. (3): the Kronecker factorisation with the shift sign reading;
* Lemma 1: Sherman-Morrison-Woodbury form and E_l^T A^{-1} E_1 = A^{-l};
* Theorem 1 / Corollary 1: spectrum of P_alpha^{-1} A;
* Fig. 2 (right): cond(U^* Gamma_alpha) = alpha^{-(l-1)/l};
* Proposition 1: Chebyshev iterate equals the polynomial T_p formula, modewise;
* Hermitian symmetry: P^{-1} r is real for real r.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import operators as ops
from oracle import precond as pc
from oracle.bounds import theorem1_eigs, cor1_interval
from synth import lognormal_kappa, random_block_vector


def _small(nx=5, ny=4, seed=0):
    kap = lognormal_kappa(nx, ny, 2.0, 2.0, 0.8, seed=seed)
    return ops.build_A(2, nx, ny, kap), kap


@pytest.mark.parametrize("ell", [2, 4, 5, 6])
@pytest.mark.parametrize("alpha", [1e-3, 1e-2, 0.5, 1.0])
def test_exact_prec_equals_dense_P_alpha(ell, alpha):
    A, _ = _small()
    P = pc.build_P_alpha(A, ell, alpha).toarray()
    r = random_block_vector(A.shape[0], ell, seed=1)
    z_dense = np.linalg.solve(P, r)
    z = pc.apply_prec_exact(A, r, ell, alpha)
    assert np.linalg.norm(z - z_dense) < 1e-12 * np.linalg.norm(z_dense)
    # the real-input preconditioner output is real (Hermitian symmetry across frequencies)
    zc = pc.apply_prec_exact(A, r, ell, alpha, return_complex=True)
    assert np.linalg.norm(zc.imag) < 1e-12 * np.linalg.norm(zc.real)


def test_literal_sign_pairing_is_wrong():
    """The printed pairing (positive-exponent shifts with the negative-exponent forward
    transform) does not invert P_alpha; the conjugated labelling does."""
    A, _ = _small()
    ell, alpha = 4, 1e-2
    n = A.shape[0]
    r = random_block_vector(n, ell, seed=2)
    z_dense = np.linalg.solve(pc.build_P_alpha(A, ell, alpha).toarray(), r)
    rhat = pc.forward_transform(r, ell, alpha)
    lam_lit = alpha ** (1 / ell) * np.exp(+2j * np.pi * np.arange(ell) / ell)
    Ad = A.toarray()
    yhat = np.array([np.linalg.solve(Ad - lam_lit[m] * np.eye(n), rhat[m]) for m in range(ell)])
    z_lit = pc.inverse_transform(yhat, ell, alpha).real
    assert np.linalg.norm(z_lit - z_dense) > 1e-2 * np.linalg.norm(z_dense)


def test_kronecker_factorisation_eq3():
    A, _ = _small(4, 3)
    ell, alpha = 5, 0.3
    n = A.shape[0]
    G = np.diag(pc.gamma(ell, alpha))
    U = pc.unitary_dft(ell)
    # The paper's U (positive-exponent columns) with the negative-exponent shifts: the
    # eigenvalue of C_alpha on Gamma^{-1} U_m is alpha^{1/l} e^{-2 pi i m / l}.
    Lam = np.diag(pc.shifts(ell, alpha))
    left = np.kron(np.linalg.inv(G) @ U, np.eye(n))
    mid = np.kron(np.eye(ell), A.toarray()) - np.kron(Lam, np.eye(n))
    right = np.kron(U.conj().T @ G, np.eye(n))
    P = pc.build_P_alpha(A, ell, alpha).toarray()
    assert np.max(np.abs(left @ mid @ right - P)) < 1e-12 * np.max(np.abs(P))
    # C_alpha = Gamma^{-1} U Lambda U^* Gamma
    C = np.linalg.inv(G) @ U @ Lam @ U.conj().T @ G
    assert np.max(np.abs(C - pc.c_alpha(ell, alpha))) < 1e-13


def test_lemma1_smw_form():
    A, _ = _small(4, 4, seed=3)
    ell, alpha = 4, 0.05
    n = A.shape[0]
    Ad = A.toarray()
    calA = ops.build_calA(A, ell).toarray()
    calAi = np.linalg.inv(calA)
    Ainv_l = np.linalg.matrix_power(np.linalg.inv(Ad), ell)
    E1 = np.kron(np.eye(ell)[:, [0]], np.eye(n))
    El = np.kron(np.eye(ell)[:, [ell - 1]], np.eye(n))
    assert np.max(np.abs(El.T @ calAi @ E1 - Ainv_l)) < 1e-13
    Z = (np.eye(n) - alpha * Ainv_l) / alpha
    Pinv = calAi + calAi @ E1 @ np.linalg.inv(Z) @ El.T @ calAi
    assert np.max(np.abs(Pinv - np.linalg.inv(pc.build_P_alpha(A, ell, alpha).toarray()))) < 1e-12


@pytest.mark.parametrize("alpha", [1e-2, 0.5])
def test_theorem1_and_corollary1(alpha):
    A, _ = _small(4, 3, seed=4)
    ell = 4
    calA = ops.build_calA(A, ell).toarray()
    P = pc.build_P_alpha(A, ell, alpha).toarray()
    ev = np.sort(np.linalg.eigvals(np.linalg.solve(P, calA)).real)
    mu = np.linalg.eigvalsh(A.toarray())
    ref = np.sort(theorem1_eigs(mu, ell, alpha))
    assert np.max(np.abs(ev - ref)) < 1e-9
    lo, hi = cor1_interval(mu.min(), ell, alpha)
    assert abs(ev.min() - lo) < 1e-9 and abs(ev.max() - hi) < 1e-9 * hi


@pytest.mark.parametrize("ell,alpha", [(4, 1e-2), (10, 1e-2), (10, 1e-4), (6, 1.0)])
def test_fig2_condition_of_eigenvector_matrix(ell, alpha):
    U = pc.unitary_dft(ell)
    G = np.diag(pc.gamma(ell, alpha))
    assert abs(np.linalg.cond(U.conj().T @ G) / alpha ** (-(ell - 1) / ell) - 1) < 1e-10


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
@pytest.mark.parametrize("dim,nx,ny", [(1, 33, 1), (2, 12, 10)])
def test_exact_closed_form_matches_direct(bc, dim, nx, ny):
    kap, ell, alpha = 6.0, 6, 1e-2
    A = ops.build_A(dim, nx, ny, kap, bc)
    r = random_block_vector(A.shape[0], ell, seed=6)
    z1 = pc.apply_prec_exact(A, r, ell, alpha)
    z2 = pc.apply_prec_closed_form(dim, nx, ny, kap, r, ell, alpha, bc=bc)
    assert np.linalg.norm(z1 - z2) < 1e-12 * np.linalg.norm(z1)


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
@pytest.mark.parametrize("p", [1, 2, 3, 7, 20])
def test_chebyshev_iterate_is_the_chebyshev_polynomial(bc, p):
    """Proposition 1: after p steps from zero, y = (1 - T_p((theta-B)/delta)/T_p(theta/delta)) B^{-1} b,
    evaluated modewise through the sine / Fourier basis (Appendix A)."""
    dim, nx, ny, kap, ell, alpha = 2, 14, 11, 9.0, 6, 0.1
    A = ops.build_A(dim, nx, ny, kap, bc)
    lo, hi = ops.constant_interval(dim, nx, ny, kap, bc)
    lo *= 0.9  # a strictly enclosing interval is as valid as the exact one
    r = random_block_vector(A.shape[0], ell, seed=7)
    pp = np.array([p, p + 1, p + 2, p, max(p - 1, 1), p])
    z_it = pc.apply_prec_nc(A, r, ell, alpha, lo, hi, pp)
    z_cf = pc.apply_prec_closed_form(dim, nx, ny, kap, r, ell, alpha, pp, lo, hi, bc=bc)
    assert np.linalg.norm(z_it - z_cf) < 1e-11 * np.linalg.norm(z_cf)


def test_nested_chebyshev_converges_to_exact():
    A, kap = _small(6, 5, seed=8)
    ell, alpha = 4, 1e-2
    lo, hi = ops.spectral_interval(2, 6, 5, kap)
    r = random_block_vector(A.shape[0], ell, seed=9)
    z_ex = pc.apply_prec_exact(A, r, ell, alpha)
    z_nc = pc.apply_prec_nc(A, r, ell, alpha, lo, hi, 400)
    assert np.linalg.norm(z_nc - z_ex) < 1e-11 * np.linalg.norm(z_ex)
    zc = pc.apply_prec_nc(A, r, ell, alpha, lo, hi, 5, return_complex=True)
    assert np.linalg.norm(zc.imag) < 1e-13 * np.linalg.norm(zc.real)


def test_chebyshev_with_initial_guess_is_affine():
    """With x_0 given, p steps give x_0 + (1 - Omega_p(B)) B^{-1} (b - B x_0): the same map
    applied to the residual of the initial guess."""
    A, kap = _small(6, 5, seed=10)
    lo, hi = ops.spectral_interval(2, 6, 5, kap)
    lam = 0.3 - 0.2j
    theta, delta = pc.cheb_centre(lo, hi, lam)
    n = A.shape[0]
    rng = np.random.default_rng(0)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    B = lambda v: A @ v - lam * v
    x = pc.chebyshev_solve(B, b, theta, delta, 6, x0)
    x_ref = x0 + pc.chebyshev_solve(B, b - B(x0), theta, delta, 6)
    assert np.linalg.norm(x - x_ref) < 1e-12 * np.linalg.norm(x_ref)
