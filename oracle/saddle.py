"""Saddle-point reformulation P_SP (Section 4) and its Krylov solvers (oracle, test
infrastructure only).

* A complex shifted system (A - lambda I) x = b with lambda = rho + i s, s != 0, is solved
  in real arithmetic (eq. (saddlesystem)).  With sigma = |s| and A - rho I SPD (mu_min >
  Re lambda), the system reads
      [[sigma I, A - rho I], [A - rho I, -sigma I]] [u1; u2] = f,
  where for s > 0: u = (Re x, -Im x), f = (-Im b, Re b), and for s < 0 (solve the
  conjugate system): u = (Re x, Im x), f = (Im b, Re b).  Both blocks of the matrix
  [[Phi, Psi], [Psi, -Phi]] are then SPD: Phi = sigma I, Psi = A - rho I.
* P_D = blkdiag(Phi + Psi, Phi + Psi) (eq. (minresprecond)); Theorem 5 puts the
  eigenvalues of P_D^{-1} S in [-1, -1/sqrt 2] U [1/sqrt 2, 1].
* Preconditioned MINRES (Paige-Saunders, in the Lanczos form with a symmetric positive
  definite preconditioner) for the saddle systems and preconditioned CG for the real
  shifts (Section 5), each for a fixed number of iterations from a zero guess; P_D and
  the CG preconditioner are applied by a V-cycle (multigrid module) or exactly.
* apply_prec_sp: eq. (4) with those inner solves for every l (conjugate pairs through
  the two branches above).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import multigrid as mg
from oracle import precond as pc


def saddle_matrix(A: sp.spmatrix, lam: complex) -> sp.csr_matrix:
    """S of eq. (saddlesystem) in the form with Phi = |Im lambda| I (see module docstring)."""
    n = A.shape[0]
    I = sp.identity(n, format="csr")
    sigma = abs(lam.imag)
    Psi = (A - lam.real * I).tocsr()
    return sp.bmat([[sigma * I, Psi], [Psi, -sigma * I]], format="csr")


def saddle_rhs(b: np.ndarray, lam: complex) -> np.ndarray:
    return np.concatenate([-b.imag, b.real]) if lam.imag > 0 else np.concatenate([b.imag, b.real])


def saddle_solution(u: np.ndarray, lam: complex) -> np.ndarray:
    n = u.shape[0] // 2
    return u[:n] - 1j * u[n:] if lam.imag > 0 else u[:n] + 1j * u[n:]


def pd_shift(lam: complex) -> float:
    """P_D's blocks are A - c I with c = Re lambda - |Im lambda|."""
    return lam.real - abs(lam.imag)


def minres(apply_S, b: np.ndarray, apply_Minv, iters: int) -> np.ndarray:
    """iters steps of preconditioned MINRES from x = 0."""
    x = np.zeros_like(b)
    v_prev = np.zeros_like(b)
    v = b.copy()
    z = apply_Minv(v)
    gamma = np.sqrt(v @ z)
    if gamma == 0.0:
        return x
    gamma_prev = 1.0
    eta = gamma
    c_prev = c = 1.0
    s_prev = s = 0.0
    w_prev = np.zeros_like(b)
    w = np.zeros_like(b)
    for _ in range(iters):
        z = z / gamma
        Sz = apply_S(z)
        delta = Sz @ z
        v_next = Sz - (delta / gamma) * v - (gamma / gamma_prev) * v_prev
        z_next = apply_Minv(v_next)
        gamma_next = np.sqrt(max(v_next @ z_next, 0.0))
        a0 = c * delta - c_prev * s * gamma
        a1 = np.hypot(a0, gamma_next)
        a2 = s * delta + c_prev * c * gamma
        a3 = s_prev * gamma
        c_prev, c = c, a0 / a1
        s_prev, s = s, gamma_next / a1
        w_next = (z - a3 * w_prev - a2 * w) / a1
        x = x + c * eta * w_next
        eta = -s * eta
        if gamma_next == 0.0:
            break
        v_prev, v = v, v_next
        w_prev, w = w, w_next
        z = z_next
        gamma_prev, gamma = gamma, gamma_next
    return x


def pcg(apply_A, b: np.ndarray, apply_Minv, iters: int) -> np.ndarray:
    """iters steps of preconditioned conjugate gradients from x = 0."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_Minv(r)
    p = z.copy()
    rho = r @ z
    for _ in range(iters):
        if rho == 0.0:
            break
        q = apply_A(p)
        a = rho / (p @ q)
        x = x + a * p
        r = r - a * q
        z = apply_Minv(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x


def shifted_solve_sp(A: sp.spmatrix, b: np.ndarray, lam: complex, iters: int, levels=None) -> np.ndarray:
    """One inner solve of (A - lambda I) x = b: CG for real lambda, saddle-point MINRES
    otherwise; preconditioner a V-cycle on `levels`, or exact when levels is None."""
    n = A.shape[0]
    I = sp.identity(n, format="csr")
    if lam.imag == 0.0:
        B = (A - lam.real * I).tocsr()
        c = lam.real
        Minv = (lambda r: mg.vcycle(levels, r, c)) if levels is not None else \
            (lambda r: spla.spsolve(B.tocsc(), r))
        return pcg(lambda v: B @ v, b.real.copy(), Minv, iters) + 0j
    S = saddle_matrix(A, lam)
    c = pd_shift(lam)
    if levels is not None:
        Minv = lambda r: np.concatenate([mg.vcycle(levels, r[:n], c), mg.vcycle(levels, r[n:], c)])
    else:
        Pd = (A - c * I).tocsc()
        Minv = lambda r: np.concatenate([spla.spsolve(Pd, r[:n]), spla.spsolve(Pd, r[n:])])
    u = minres(lambda v: S @ v, saddle_rhs(b, lam), Minv, iters)
    return saddle_solution(u, lam)


def apply_prec_sp(A: sp.spmatrix, r: np.ndarray, ell: int, alpha: float, iters: int, levels=None,
                  return_complex: bool = False):
    """P_SP^{-1} r: eq. (4) with every shifted solve done by shifted_solve_sp."""
    rhat = pc.forward_transform(r, ell, alpha)
    lam = pc.shifts(ell, alpha)
    yhat = np.empty_like(rhat)
    for m in range(ell):
        lm = complex(lam[m])
        if m == 0 or (ell % 2 == 0 and m == ell // 2):
            lm = complex(lm.real, 0.0)  # the real shifts, without the polar form's residue
        yhat[m] = shifted_solve_sp(A, rhat[m], lm, iters, levels)
    y = pc.inverse_transform(yhat, ell, alpha)
    return y if return_complex else y.real
