"""Outer solvers for the all-at-once system, FP64.

* ``fgmres``: right-preconditioned flexible GMRES(m).  Arnoldi by classical
  Gram-Schmidt applied twice (CGS2), Givens rotations on the Hessenberg matrix,
  x = x_0 + Z y with Z the stored preconditioned vectors.  With a linear
  preconditioner this is right-preconditioned GMRES.  The stopping test uses the
  true relative residual ||b - A x|| / ||b|| (the paper's definition of the
  relative residual, Section 5): when the Givens estimate reaches the tolerance,
  the iterate is formed and its true residual checked; if that is not yet below
  the tolerance the cycle restarts from the iterate.  The outer Krylov method is
  not the paper's (which uses Chebyshev semi-iteration); it has no paper pin and
  is checked against direct solves.
* ``outer_chebyshev``: the paper's outer method, Chebyshev semi-iteration on
  P^{-1} A with the Corollary 1 interval, x_0 = 0, stopped when the relative
  residual falls below the tolerance (Section 2, Section 5; the bounds are not
  adjusted for an approximate P).  Pinned by the NC2 outer counts of Table 3.
"""

from __future__ import annotations

import numpy as np


def fgmres(apply_op, b: np.ndarray, apply_prec=None, tol: float = 1e-8, m: int = 30, max_outer: int = 1000,
           x0=None):
    """Returns (x, info) with info = {iterations, restarts, rel_residual, history}."""
    prec = apply_prec if apply_prec is not None else (lambda v: v.copy())
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    history = []
    if bnorm == 0.0:
        return np.zeros_like(b), {"iterations": 0, "restarts": 0, "rel_residual": 0.0, "history": history}
    r = b - apply_op(x)
    beta = np.linalg.norm(r)
    total = 0
    restarts = 0
    while True:
        if beta / bnorm <= tol or total >= max_outer:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k_done = 0
        for j in range(m):
            z = prec(V[j])
            Z.append(z)
            w = apply_op(z)
            # CGS2: two passes of classical Gram-Schmidt
            h = np.zeros(j + 1)
            for _ in range(2):
                Vm = np.array(V)
                c = Vm @ w
                w = w - Vm.T @ c
                h += c
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k_done = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or total >= max_outer or hn == 0.0:
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + np.array(Z).T @ y
        r = b - apply_op(x)
        beta = np.linalg.norm(r)
        restarts += 1
    return x, {"iterations": total, "restarts": restarts, "rel_residual": beta / bnorm, "history": history}


def outer_chebyshev(apply_op, b: np.ndarray, apply_prec, lo: float, hi: float, tol: float = 1e-6,
                    max_iter: int = 10000):
    """Preconditioned Chebyshev semi-iteration with eigenvalue interval [lo, hi] of
    P^{-1} A, x_0 = 0, stopped on ||b - A x_k|| / ||b|| < tol.  Returns (x, iterations)
    where iterations counts the updates x_{k+1} = x_k + d_k that were taken."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_prec(r)
    d = z / theta
    rho = delta / theta
    it = 0
    while it < max_iter:
        x = x + d
        it += 1
        r = b - apply_op(x)
        if np.linalg.norm(r) / bnorm < tol:
            break
        z = apply_prec(r)
        rho_next = 1.0 / (2.0 * theta / delta - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * z
        rho = rho_next
    return x, it
