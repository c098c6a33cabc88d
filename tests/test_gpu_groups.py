"""Steady sweeps in shift groups (at most one real and two complex shifts per
launch) compute exactly what the all-shift sweep computes: P_NC^{-1} with and
without grouping, for even and odd l, uniform and NC2 (uneven, some shifts finished
early) inner counts, and both precisions; plus the oracle at one point."""

import numpy as np
import pytest

from oracle import operators as ops
from oracle import precond as pc
from paper_2506_03947_amd import api
from synth import lognormal_kappa
from tests import gpu_util as G

L = api.L
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ell", [5, 8, 10, 12, 16])
@pytest.mark.parametrize("precision", [L.AC_PREC_FP64, L.AC_PREC_MIXED_BF16K])
@pytest.mark.parametrize("nc2", [False, True])
def test_grouped_sweeps_equal_all_shift_sweeps(ell, precision, nc2):
    nx, ny = 200, 75
    kap = lognormal_kappa(nx, ny, 20.0, 6.0, 1.0, seed=ell)
    p = G.problem(2, nx, ny, kap, ell, 1e-2)
    pm = api.ac_alloc_nc2(p, 7.0 * ell) if nc2 else 7
    opts = api.Opts(precision=precision, p=pm)
    ws = api.workspace(api.ac_prec_workspace_size(p, opts))
    r = G.dev(np.random.default_rng(ell).standard_normal(ell * nx * ny))
    out = []
    api.ac_ctx_set_step_pairs(G.ctx(), 0)  # single steady steps: grouped or all-shift
    try:
        for mode in (0, 1):
            api.ac_ctx_set_shift_groups(G.ctx(), mode)
            z = G.dev(np.zeros(ell * nx * ny))
            api.ac_apply_prec(p, opts, r, z, ws)
            out.append(G.host(z))
    finally:
        api.ac_ctx_set_shift_groups(G.ctx(), -1)
        api.ac_ctx_set_step_pairs(G.ctx(), 1)
    # float32: another kernel variant may contract operations differently; a few
    # roundings (2^-24) per step, amplified by cond(U* Gamma) = alpha^{-(l-1)/l}
    tol = 1e-14 if precision == L.AC_PREC_FP64 else 8 * 7 * 1e-2 ** (-(ell - 1) / ell) * 2.0 ** -24
    assert G.max_rel(out[1], out[0]) <= tol
    if precision == L.AC_PREC_FP64 and ell == 10 and nc2:
        A = ops.build_A(2, nx, ny, kap)
        lo, hi = api.ac_spectral_bounds(p)
        ref = pc.apply_prec_nc(A, G.host(r), ell, 1e-2, lo, hi, pm)
        assert G.rel(out[1], ref) < 1e-12
