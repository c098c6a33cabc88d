"""Inner Chebyshev counts of Table 2 on the GPU: for the paper operator (n_x = 100, l = 10,
alpha = 1) and each of the six distinct shifts, the library's shifted Chebyshev solve
reaches the relative residual eps after exactly the number of steps the oracle's iteration
needs (the oracle's counts are pinned to the paper's Table 2 in
tests/test_oracle_bounds_alloc.py)."""

import numpy as np
import pytest
import torch

from oracle import operators as ops
from oracle import precond as pc
from oracle.alloc import paper_operator_kappa
from paper_2506_03947_amd import api
from tests import gpu_util as G

L = api.L
pytestmark = pytest.mark.gpu


def _oracle_counts(A, lams, lo, hi, b, eps_list, maxit=2000):
    """Steps of Chebyshev semi-iteration (residual form, zero start) until the relative
    residual falls below each eps."""
    out = []
    for lam in lams:
        theta, delta = pc.cheb_centre(lo, hi, lam)
        x = np.zeros_like(b, dtype=complex)
        r = b.astype(complex)
        bn = np.linalg.norm(b)
        rho = delta / theta
        d = r / theta
        res = {}
        for k in range(maxit):
            x = x + d
            r = r - (A @ d - lam * d)
            rel = np.linalg.norm(r) / bn
            for e in eps_list:
                if e not in res and rel < e:
                    res[e] = k + 1
            if len(res) == len(eps_list):
                break
            rn = 1 / (2 * theta / delta - rho)
            d = rn * rho * d + (2 * rn / delta) * r
            rho = rn
        out.append(res)
    return out


def test_table2_inner_counts_gpu():
    nx, ell, alpha = 100, 10, 1.0
    kap = paper_operator_kappa(nx, ell)
    lo, hi = ops.constant_interval(2, nx, nx, kap)
    A = ops.build_A(2, nx, nx, kap)
    lam = pc.shifts(ell, alpha)
    eps_list = [1e-10, 1e-6, 1e-1]
    b = np.ones(nx * nx)
    counts = _oracle_counts(A, lam[:6], lo, hi, b, eps_list)
    p = G.problem(2, nx, nx, kap, ell, alpha, bounds=(lo, hi))
    rbuf = api.complex_to_spectral(p, 0, [torch.ones(p.n, dtype=torch.complex128, device="cuda:0")
                                          for _ in range(p.ns)])
    ybuf = torch.zeros_like(rbuf)

    def residuals(steps):
        """True relative residuals |b - (A - lambda_m I) y_m| / |b| of the GPU's float64
        solutions, formed on the host with the oracle's A."""
        pm = [steps[min(m, ell - m)] for m in range(ell)]
        opts = api.Opts(precision=L.AC_PREC_FP64, p=pm)
        api.ac_shifted_cheb(p, opts, rbuf, None, ybuf, api.workspace(api.ac_prec_workspace_size(p, opts)))
        ys = [G.host(t) for t in api.spectral_to_complex(p, 0, ybuf)]
        return np.array([np.linalg.norm(b - (A @ ys[m] - lam[m] * ys[m])) / np.linalg.norm(b) for m in range(6)])

    for e in eps_list:
        c = [counts[m][e] for m in range(6)]
        print(f"eps {e:g}: oracle counts {c}", flush=True)
        at = residuals([ci + 1 for ci in c])
        assert np.all(at < e), (e, at)
        below = residuals([max(ci - 2, 1) for ci in c])
        for m in range(6):
            if c[m] > 2:
                assert below[m] > e, (e, m, below[m])
