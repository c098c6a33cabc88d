"""Block alpha-circulant preconditioner: exact and nested-Chebyshev applications.

Definitions followed (Section 2, Section 2.2, Section 3):
* P_alpha = I_l (x) A - C_alpha (x) I_N, with C_alpha the down-shift carrying
  alpha in its top-right corner (eq. (2)).
* Gamma_alpha = diag(alpha^{(k-1)/l}), k = 1..l (Section 2.2).
* P_alpha^{-1} = (Gamma^{-1} U (x) I)(I (x) A - Lambda (x) I)^{-1}(U^* Gamma (x) I)
  (eq. (4)), so applying it is: scale by Gamma, DFT across the blocks, l shifted
  solves (A - lambda_j I) y_j = r_j (eq. (6)), inverse DFT, scale by Gamma^{-1}.

Reading of the DFT sign (the printed pairing of U and Lambda in eq. (3) is
inconsistent with C_alpha being a down-shift): the down-shift maps the Fourier
vector (e^{+2 pi i m k / l})_k to e^{-2 pi i m / l} times itself, so with the
forward transform taken with the negative exponent (numpy's fft) the shift
paired with frequency m is lambda_m = alpha^{1/l} e^{-2 pi i m / l}.  The set of
shifts is the paper's; only the labelling is conjugated.  The dense brute-force
check of P_alpha (tests) decides this reading.

Nested Chebyshev (Section 3): each shifted system is solved by p_j steps of
Chebyshev semi-iteration on the segment S_j = [mu_lo - lambda_j, mu_hi - lambda_j]
(Lemma 2), i.e. the limit case E_j = S_j, whose error polynomial is
T_p((theta_j - z)/delta)/T_p(theta_j/delta) with centre theta_j =
(mu_hi + mu_lo)/2 - lambda_j and half-width delta = (mu_hi - mu_lo)/2
(Proposition 1).  The recurrence is the textbook residual/direction form of
Chebyshev acceleration (Axelsson 1996 Sec. 5.3; Saad, Iterative Methods,
Alg. 12.1) with a complex centre; the paper does not print it.

Pins: dense P_alpha from eq. (2) on tiny N; Lemma 1 (SMW) form; Theorem 1
spectrum; Fig. 2 (right) conditioning of U^* Gamma; closed-form modewise
multipliers for constant coefficients; Proposition 1 per-step bound.
"""

from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import dirichlet_eigs, periodic_eigs


def shifts(ell: int, alpha: float) -> np.ndarray:
    """lambda_m = alpha^{1/l} exp(-2 pi i m / l), m = 0..l-1 (see module docstring)."""
    m = np.arange(ell)
    return alpha ** (1.0 / ell) * np.exp(-2j * np.pi * m / ell)


def gamma(ell: int, alpha: float) -> np.ndarray:
    """Diagonal of Gamma_alpha: alpha^{(k-1)/l}, k = 1..l (Section 2.2)."""
    return alpha ** (np.arange(ell) / ell)


def c_alpha(ell: int, alpha: float) -> np.ndarray:
    """Dense C_alpha of eq. (2): ones below the diagonal, alpha in the top-right corner."""
    C = np.diag(np.ones(ell - 1), -1)
    C[0, ell - 1] = alpha
    return C


def build_P_alpha(A: sp.spmatrix, ell: int, alpha: float) -> sp.csr_matrix:
    """Explicit P_alpha = I (x) A + C_alpha (x) (-I) of eq. (2)."""
    n = A.shape[0]
    return (sp.kron(sp.identity(ell), A) - sp.kron(sp.csr_matrix(c_alpha(ell, alpha)), sp.identity(n))).tocsr()


def unitary_dft(ell: int) -> np.ndarray:
    """U with columns (1/sqrt(l)) (exp(2 pi i (j-1)(k-1)/l))_k (Section 2.2)."""
    k = np.arange(ell)
    return np.exp(2j * np.pi * np.outer(k, k) / ell) / np.sqrt(ell)


def forward_transform(r: np.ndarray, ell: int, alpha: float) -> np.ndarray:
    """rhat = (F Gamma (x) I) r with F the unnormalised DFT (negative exponent) over the
    block index; returns an (l, N) complex array, row m paired with shift lambda_m."""
    n = r.size // ell
    R = r.reshape(ell, n) * gamma(ell, alpha)[:, None]
    return np.fft.fft(R, axis=0)


def inverse_transform(yhat: np.ndarray, ell: int, alpha: float) -> np.ndarray:
    """y = (Gamma^{-1} F^{-1} (x) I) yhat (complex, length l*N)."""
    Y = np.fft.ifft(yhat, axis=0) / gamma(ell, alpha)[:, None]
    return Y.reshape(-1)


def apply_prec_exact(A: sp.spmatrix, r: np.ndarray, ell: int, alpha: float, return_complex: bool = False):
    """Exact P_alpha^{-1} r by l sparse LU solves of (A - lambda_m I) (eq. (4), eq. (6))."""
    n = A.shape[0]
    rhat = forward_transform(r, ell, alpha)
    lam = shifts(ell, alpha)
    I = sp.identity(n, format="csc")
    yhat = np.empty_like(rhat)
    Acsc = A.tocsc().astype(np.complex128)
    for m in range(ell):
        lu = spla.splu((Acsc - lam[m] * I).tocsc())
        yhat[m] = lu.solve(rhat[m])
    y = inverse_transform(yhat, ell, alpha)
    return y if return_complex else y.real


def chebyshev_solve(apply_B, b: np.ndarray, theta: complex, delta: float, p: int, x0=None) -> np.ndarray:
    """p steps of Chebyshev semi-iteration for B x = b on the segment theta +- delta.

    Residual/direction form: r_0 = b - B x_0, rho_0 = delta/theta, d_0 = r_0/theta;
    x_{k+1} = x_k + d_k; r_{k+1} = r_k - B d_k; rho_{k+1} = 1/(2 theta/delta - rho_k);
    d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) r_{k+1}.
    After p steps e_p = T_p((theta - B)/delta) / T_p(theta/delta) e_0.
    """
    x = np.zeros_like(b, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    if p <= 0:
        return x
    r = b.astype(np.complex128) - (apply_B(x) if x0 is not None else 0.0)
    rho = delta / theta
    d = r / theta
    for k in range(p):
        x = x + d
        if k == p - 1:
            break
        r = r - apply_B(d)
        rho_next = 1.0 / (2.0 * theta / delta - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * r
        rho = rho_next
    return x


def cheb_centre(mu_lo: float, mu_hi: float, lam: complex):
    """Centre theta_j = (mu_hi + mu_lo)/2 - lambda_j and half-width delta of S_j (Lemma 2)."""
    return 0.5 * (mu_hi + mu_lo) - lam, 0.5 * (mu_hi - mu_lo)


def apply_prec_nc(A: sp.spmatrix, r: np.ndarray, ell: int, alpha: float, mu_lo: float, mu_hi: float,
                  p_per_shift, x0_hat=None, return_complex: bool = False, workers: int = 1):
    """Nested-Chebyshev P_NC^{-1} r: eq. (4) with every shifted solve replaced by p_m
    Chebyshev steps (Section 3).  ``p_per_shift[m]`` pairs with lambda_m; ``x0_hat``
    optionally gives per-shift initial guesses (an (l, N) complex array); ``workers``
    > 1 runs the l independent shifted solves on a thread pool (same arithmetic)."""
    n = A.shape[0]
    rhat = forward_transform(r, ell, alpha)
    lam = shifts(ell, alpha)
    p = np.broadcast_to(np.asarray(p_per_shift, dtype=int), (ell,))
    yhat = np.empty_like(rhat)

    def solve_shift(m):
        theta, delta = cheb_centre(mu_lo, mu_hi, lam[m])
        lm = lam[m]

        def apply_B(v):
            return A @ v - lm * v

        yhat[m] = chebyshev_solve(apply_B, rhat[m], theta, delta, int(p[m]),
                                  None if x0_hat is None else x0_hat[m])

    if workers > 1:
        # the shifted solves are independent; each runs whole on one thread
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(solve_shift, range(ell)))
    else:
        for m in range(ell):
            solve_shift(m)
    y = inverse_transform(yhat, ell, alpha)
    return y if return_complex else y.real


def chebyshev_T(p: int, z):
    """T_p(z) for complex z via T_p = ((z + s)^p + (z - s)^p)/2, s = sqrt(z^2 - 1) taken
    with positive real part (proof of Theorem 4)."""
    z = np.asarray(z, dtype=np.complex128)
    s = np.sqrt(z * z - 1.0)
    s = np.where(s.real < 0, -s, s)
    return 0.5 * ((z + s) ** p + (z - s) ** p)


def cheb_multiplier(xi, theta: complex, delta: float, p: int):
    """Modewise action of p Chebyshev steps from x_0 = 0 on an eigenvalue xi of B:
    y = (1 - Omega_p(xi)) / xi * b with Omega_p(xi) = T_p((theta - xi)/delta)/T_p(theta/delta)
    (Proposition 1).  T_p is evaluated by the three-term recurrence."""
    xi = np.asarray(xi, dtype=np.complex128)
    z = (theta - xi) / delta
    z0 = theta / delta
    t_prev, t = np.ones_like(z), z.copy()
    s_prev, s = 1.0 + 0j, z0
    if p == 0:
        return np.zeros_like(xi)
    for _ in range(p - 1):
        t_prev, t = t, 2.0 * z * t - t_prev
        s_prev, s = s, 2.0 * z0 * s - s_prev
    return (1.0 - t / s) / xi


def _mode_transform(dim: int, nx: int, ny: int, bc: str):
    """Orthonormal spatial transform diagonalising a constant-coefficient A:
    DST-I per axis (Dirichlet; sine vectors of Appendix A) or the unitary FFT (periodic)."""
    shape = (nx,) if dim == 1 else (ny, nx)
    axes = (0,) if dim == 1 else (0, 1)
    if bc == "dirichlet":
        fwd = lambda v: sfft.dstn(v.reshape(shape), type=1, axes=axes, norm="ortho")
        inv = lambda v: sfft.idstn(v, type=1, axes=axes, norm="ortho").reshape(-1)
    else:
        fwd = lambda v: sfft.fftn(v.reshape(shape), axes=axes, norm="ortho")
        inv = lambda v: sfft.ifftn(v, axes=axes, norm="ortho").reshape(-1)
    return fwd, inv


def apply_prec_closed_form(dim: int, nx: int, ny: int, kappa: float, r: np.ndarray, ell: int, alpha: float,
                           p_per_shift=None, mu_lo: float | None = None, mu_hi: float | None = None,
                           bc: str = "dirichlet", return_complex: bool = False):
    """Constant-coefficient P_alpha^{-1} (p_per_shift None) or P_NC^{-1} at any N in
    O(l N log N): spatial DST-I / FFT diagonalises A (Appendix A), so each shifted solve
    is a per-mode multiplier 1/xi (exact) or cheb_multiplier (nested CI)."""
    n = nx * (ny if dim == 2 else 1)
    mu = dirichlet_eigs(dim, nx, ny, kappa) if bc == "dirichlet" else periodic_eigs(dim, nx, ny, kappa)
    fwd, inv = _mode_transform(dim, nx, ny, bc)
    rhat = forward_transform(r, ell, alpha)
    lam = shifts(ell, alpha)
    yhat = np.empty((ell, n), dtype=np.complex128)
    for m in range(ell):
        xi = mu - lam[m]
        if p_per_shift is None:
            mult = 1.0 / xi
        else:
            theta, delta = cheb_centre(mu_lo, mu_hi, lam[m])
            mult = cheb_multiplier(xi, theta, delta, int(np.broadcast_to(p_per_shift, (ell,))[m]))
        yhat[m] = inv(mult * fwd(rhat[m]))
    y = inverse_transform(yhat, ell, alpha)
    return y if return_complex else y.real
