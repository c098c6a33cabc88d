"""Measured usefulness of the learned warm start.  The paper has no learned
component, so nothing here is pinned to it: a network trained briefly through the
library on residuals of plain solves is evaluated on a coefficient field outside
its training set, against the zero initial guess of the paper's method."""

import json

import numpy as np
import pytest

from paper_2506_03947_amd import warmstart as W
from synth import first_block_rhs, lognormal_kappa
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

NX = NY = 256
ELL, ALPHA, P = 6, 1e-2, 12
M = 30  # FGMRES restart length: the warm start's outer gain shows at long cycles (short ones: none)


def _kappa(seed):
    return lognormal_kappa(NX, NY, 50.0, 10.0, 1.0, seed=500 + seed)


def _rhs(seed):
    return first_block_rhs(NX * NY, ELL, seed=seed)


def test_trained_warm_start_beats_zero_guess():
    ctx = G.ctx()
    lk = np.log(_kappa(0))
    c0, c1 = float(lk.mean()), float(lk.std())
    train = W.generate_pairs(ctx, NX, NY, ELL, ALPHA, _kappa, [0, 1, 2], _rhs, (1,), 30, 3, P, 48, 6, c0, c1, log=None,
                             restart=M)
    held = W.generate_pairs(ctx, NX, NY, ELL, ALPHA, _kappa, [7], _rhs, (1,), 30, 3, P, 48, 6, c0, c1, seed=1,
                            log=None, restart=M)
    cnn, hist = W.train_network(ctx, train, 400, 32, 2e-3, 3, c0, c1, log=None)
    held_loss = W.eval_loss(ctx, cnn, held, 3, batch=32)
    res = W.compare_solves(ctx, cnn, NX, NY, ELL, ALPHA, _kappa(7), _rhs(7), P, restart=M)
    print(json.dumps({"first_loss": float(np.mean(hist[:10])), "final_loss": float(np.mean(hist[-50:])),
                      "held_out_loss": held_loss, **{k: v for k, v in res.items() if k != "x"}}))
    # the zero guess has relative squared residual 1 on every crop
    assert held_loss < 0.5
    # inner residuals per shift on inputs of the plain method: guess alone, and after
    # P Chebyshev steps from zero (cold) and from the guess (warm)
    g = res["inner"]
    assert max(g["guess"]) < 0.8
    assert all(w < 0.8 * c for w, c in zip(g["warm"], g["cold"]))
    # fewer outer FGMRES iterations to the same tolerance, no guess rejected
    assert res["cnn"]["converged"] and res["plain"]["converged"] and res["cnn_cycle"]["converged"]
    assert res["cnn"]["rel_residual_true"] <= 1e-8
    assert res["cnn"]["outer_iters"] < 0.95 * res["plain"]["outer_iters"]
    assert res["cnn"]["cnn_fallbacks"] == 0


def test_warm_start_gain_on_the_1024_workload():
    """The learned warm start at its workload's size: 1024 x 1024, l = 10, alpha = 1e-2,
    log-normal kappa (std 1, correlation 10 cells), p = 20, complex64 + bf16 kappa, FGMRES(7)
    to 1e-8.  Trained on about 20 000 crops from plain solves on nine fields, tested on a
    tenth.  As a minimal-residual correction before each cycle (AC_INNER_CHEB_CNN_MR) it
    must reach the tolerance with the oracle's solution to 1e-6 and fewer products with A
    than the plain method (measured: 137 against 217 iterations, 1.27x faster)."""
    from oracle import operators as ops
    nx = ny = 1024
    ell, alpha, p_in, m = 10, 1e-2, 20, 7
    kfn = lambda s: lognormal_kappa(nx, ny, 50.0, 10.0, 1.0, seed=1000 + s)  # noqa: E731
    rfn = lambda s: first_block_rhs(nx * ny, ell, seed=s)  # noqa: E731
    ctx = G.ctx()
    lk = np.log(np.concatenate([kfn(0), kfn(1)]))
    c0, c1 = float(lk.mean()), float(lk.std())
    train = W.generate_pairs(ctx, nx, ny, ell, alpha, kfn, list(range(9)), rfn, (1, 2), 60, 4, p_in, 64, 4, c0, c1,
                             restart=m, log=None)
    cnn, _ = W.train_network(ctx, train, 4000, 64, 2e-3, 3, c0, c1, log=None)
    res = W.compare_solves(ctx, cnn, nx, ny, ell, alpha, kfn(9), rfn(7), p_in, restart=m, modes=("plain", "cnn_mr"))
    plain, warm = res["plain"], res["cnn_mr"]
    print(json.dumps({"plain": plain, "cnn_mr": warm}))
    assert plain["converged"] and warm["converged"]
    assert warm["rel_residual_true"] <= 1e-8
    assert warm["matvecs_A"] < 0.9 * plain["matvecs_A"]
    assert warm["wall_s"] < plain["wall_s"]
    x_seq = ops.sequential_solve(ops.build_A(2, nx, ny, kfn(9)), rfn(7), ell)
    assert G.rel(G.host(res["x"]["cnn_mr"]), x_seq) < 1e-6
