"""Inner-iteration allocation: NC1 (uniform) and NC2 (Algorithm 1), Section 5.1.

Algorithm 1: for every shift compute the real-part factor
sigma_j = (sqrt(kappa_j) - 1)/(sqrt(kappa_j) + 1) with kappa_j the condition number
of Re(B_j) = A - Re(lambda_j) I, i.e. (mu_hi - Re lambda_j)/(mu_lo - Re lambda_j);
r(j) = ln(sigma_1)/ln(sigma_j); normalise r to sum one; the allocation is
floor(r * budget) entrywise, with budget = l * n_x * eta (Table 1).

Reading: the floor can give zero for a shift, which would drop a frequency and
make the preconditioner singular, so every entry is clamped to at least one.
Published rows never hit the clamp.

Pin: l + sum(allocation) equals the matvecs-per-iteration ratio of every NC2
entry of Tables 3, 4 and 8 (tests/golden/nc2_tables.json).
"""

from __future__ import annotations

import numpy as np

from .precond import shifts


def sigma_real_part(mu_lo: float, mu_hi: float, re_lam: float) -> float:
    """sigma_j of Theorem 4 from the condition number of Re(B_j)."""
    kap = (mu_hi - re_lam) / (mu_lo - re_lam)
    s = np.sqrt(kap)
    return (s - 1.0) / (s + 1.0)


def alg1_allocation(ell: int, budget: float, mu_lo: float, mu_hi: float, alpha: float) -> np.ndarray:
    """Algorithm 1 (NC2).  Entry m pairs with shift lambda_m of ``precond.shifts``; the
    allocation depends on Re(lambda) only, so the conjugate labelling does not matter."""
    lam = shifts(ell, alpha)
    sig = np.array([sigma_real_part(mu_lo, mu_hi, l.real) for l in lam])
    r = np.log(sig[0]) / np.log(sig)
    r = r / r.sum()
    alloc = np.floor(r * budget).astype(int)
    return np.maximum(alloc, 1)


def nc1_allocation(ell: int, budget: float) -> np.ndarray:
    """NC1: the same number of inner iterations, floor(budget / l), for every shift."""
    return np.full(ell, max(int(np.floor(budget / ell)), 1), dtype=int)


def paper_operator_kappa(nx: int, ell: int, D: float = 0.2) -> float:
    """Coefficient kappa = nu / h^2 of the paper's operator A = I - (nu/h^2) L, with
    nu = D^2/(2 l - 4) and h = 1/(n_x + 1) (Section 5, eq. (IminusLap))."""
    nu = D * D / (2 * ell - 4)
    h = 1.0 / (nx + 1)
    return nu / (h * h)
