"""Scalar convergence bounds of Sections 2 and 3.

* Corollary 1: for 0 < alpha < mu_min^l the spectrum of P_alpha^{-1} A lies in
  [1, mu_min^l / (mu_min^l - alpha)].
* Remark 1: for alpha <= eta < 1, max |lambda - 1| <= alpha / (1 - eta).
* Theorem 3 (Axelsson): CI on an SPD matrix with spectrum in [v_min, v_max]
  reaches tolerance eps in ceil(p*) steps,
  p* = ln(1/eps + sqrt(1/eps^2 - 1)) / ln((1 + sqrt(v_min/v_max)) / (1 - sqrt(v_min/v_max))).
* Proposition 1: ||e_p|| / ||e_0|| <= 1 / |T_p(theta_j/delta)|.
* Lemma 3 / Theorem 4: asymptotic factor rho(lambda_j) <= 1/|z + sqrt(z^2-1)| with
  z = theta_j/delta, and this is strictly below sigma_j computed from Re(lambda_j).
"""

from __future__ import annotations

import numpy as np

from .precond import chebyshev_T


def cor1_interval(mu_min: float, ell: int, alpha: float):
    """Extreme eigenvalues of P_alpha^{-1} A (Corollary 1)."""
    m = mu_min ** ell
    return 1.0, m / (m - alpha)


def theorem1_eigs(mu: np.ndarray, ell: int, alpha: float) -> np.ndarray:
    """Theorem 1: 1 with multiplicity (l-1)N, plus mu_j^l/(mu_j^l - alpha)."""
    n = mu.size
    return np.concatenate([np.ones((ell - 1) * n), mu ** ell / (mu ** ell - alpha)])


def axelsson_pstar(eps: float, v_min: float, v_max: float) -> float:
    """Theorem 3."""
    q = np.sqrt(v_min / v_max)
    return np.log(1.0 / eps + np.sqrt(1.0 / eps ** 2 - 1.0)) / np.log((1.0 + q) / (1.0 - q))


def prop1_bound(theta: complex, delta: float, p: int) -> float:
    """Proposition 1 per-step error bound 1/|T_p(theta/delta)|."""
    return float(1.0 / abs(chebyshev_T(p, theta / delta)))


def lemma3_factor(theta: complex, delta: float) -> float:
    """Lemma 3 limit: 1/|z + sqrt(z^2 - 1)|, z = theta/delta, positive-real-part root."""
    z = complex(theta / delta)
    s = np.sqrt(z * z - 1.0)
    if s.real < 0:
        s = -s
    return float(1.0 / abs(z + s))


def theorem4_sigma(mu_lo: float, mu_hi: float, re_lam: float) -> float:
    """sigma_j of Theorem 4 (condition number of Re(B_j))."""
    k = (mu_hi - re_lam) / (mu_lo - re_lam)
    return float((np.sqrt(k) - 1.0) / (np.sqrt(k) + 1.0))
