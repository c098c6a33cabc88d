"""Batched solves of independent problems with uneven grids and l: every problem's
solution against the sequential oracle and against its own single-problem solve;
convergence masking keeps early finishers fixed while the others iterate (the
captured per-iteration graphs are replayed many times with eager Krylov work in
between, and every replay feeds the checked results)."""

import numpy as np
import pytest
import torch

from oracle import operators as ops
from paper_2506_03947_amd import api
from synth import first_block_rhs, lognormal_kappa
from tests import gpu_util as G

L = api.L
pytestmark = pytest.mark.gpu

# (nx, ny, l, alpha, kappa0): uneven sizes, odd and even l, one grid too narrow for
# two points per lane, one ragged against the 16-row chunks
CASES = [(96, 64, 4, 1e-2, 20.0), (130, 70, 6, 1e-1, 10.0), (64, 50, 5, 1e-2, 30.0), (160, 96, 8, 1e-2, 50.0),
         (40, 33, 3, 1e-3, 5.0), (256, 128, 10, 1e-2, 50.0)]


def _problems(cases, seed0=0):
    probs, kaps, bs = [], [], []
    for i, (nx, ny, ell, alpha, k0) in enumerate(cases):
        kap = lognormal_kappa(nx, ny, k0, 5.0, 1.0, seed=seed0 + i)
        probs.append(G.problem(2, nx, ny, kap, ell, alpha))
        kaps.append(kap)
        bs.append(first_block_rhs(nx * ny, ell, seed=100 + i))
    return probs, kaps, bs


@pytest.mark.parametrize("precision", [L.AC_PREC_FP64, L.AC_PREC_MIXED_BF16K])
def test_batch_matches_single_and_oracle(precision):
    probs, kaps, bs = _problems(CASES)
    opts = api.Opts(precision=precision, p=8, tol=1e-10, restart_m=12, max_outer=800)
    ws = api.workspace(api.ac_batch_workspace_size(G.ctx(), probs, opts))
    xs = [G.dev(np.zeros_like(b)) for b in bs]
    infos = api.ac_batch_solve(G.ctx(), probs, opts, [G.dev(b) for b in bs], xs, ws)
    for i, (p, kap, b, info, x) in enumerate(zip(probs, kaps, bs, infos, xs)):
        nx, ny, ell = CASES[i][:3]
        assert info["converged"] and info["rel_residual_true"] <= 1e-10, (i, info)
        A = ops.build_A(2, nx, ny, kap)
        ref = ops.sequential_solve(A, b, ell)
        assert G.rel(G.host(x), ref) < 1e-6, i
        # the same problem alone: same arithmetic per kernel, so the same iterations
        x1 = G.dev(np.zeros_like(b))
        w1 = api.workspace(api.ac_solve_workspace_size(p, opts))
        one = api.ac_solve(p, opts, G.dev(b), x1, w1)
        assert abs(one["outer_iters"] - info["outer_iters"]) <= 2, (i, one, info)
        assert G.rel(G.host(x), G.host(x1)) < 1e-8, i


def test_batch_masks_converged_problems():
    """A problem with a zero right-hand side finishes at once, one with a loose
    tolerance reached early stays untouched while the others continue."""
    probs, kaps, bs = _problems(CASES[:3], seed0=10)
    bs[1] = np.zeros_like(bs[1])
    opts = api.Opts(precision=L.AC_PREC_MIXED_FP32K, p=6, tol=1e-9, restart_m=8, max_outer=600)
    ws = api.workspace(api.ac_batch_workspace_size(G.ctx(), probs, opts))
    xs = [G.dev(np.full_like(b, 3.0)) for b in bs]
    infos = api.ac_batch_solve(G.ctx(), probs, opts, [G.dev(b) for b in bs], xs, ws)
    assert infos[1]["outer_iters"] == 0 and not G.host(xs[1]).any()
    for i in (0, 2):
        nx, ny, ell = CASES[i][:3]
        ref = ops.sequential_solve(ops.build_A(2, nx, ny, kaps[i]), bs[i], ell)
        assert infos[i]["converged"] and G.rel(G.host(xs[i]), ref) < 1e-6


def test_batch_errors():
    probs, _, bs = _problems(CASES[:2])
    opts = api.Opts(precision=L.AC_PREC_FP64, p=[4] * CASES[0][2], tol=1e-8)
    with pytest.raises(api.L.AlphacircError):
        api.ac_batch_workspace_size(G.ctx(), probs, opts)
    opts = api.Opts(precision=L.AC_PREC_FP64, p=4, tol=1e-8)
    with pytest.raises(api.L.AlphacircError):
        api.ac_batch_solve(G.ctx(), probs, opts, [G.dev(b) for b in bs], [G.dev(np.zeros_like(b)) for b in bs],
                           api.workspace(1024))
