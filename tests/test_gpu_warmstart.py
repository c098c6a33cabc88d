"""Measured usefulness of the learned warm start.  The paper has no learned
component, so nothing here is pinned to it: a network trained briefly through the
library on residuals of plain solves is evaluated on a coefficient field outside
its training set, against the zero initial guess of the paper's method."""

import json

import numpy as np
import pytest

from paper_2506_03947_amd import warmstart as W
from synth import lognormal_kappa
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

NX = NY = 256
ELL, ALPHA, P = 6, 1e-2, 12
M = 30  # FGMRES restart length: the warm start's outer gain shows at long cycles (short ones: none)


def _kappa(seed):
    return lognormal_kappa(NX, NY, 50.0, 10.0, 1.0, seed=500 + seed)


def test_trained_warm_start_beats_zero_guess():
    ctx = G.ctx()
    lk = np.log(_kappa(0))
    c0, c1 = float(lk.mean()), float(lk.std())
    train = W.generate_pairs(ctx, NX, NY, ELL, ALPHA, _kappa, [0, 1, 2], (1,), 30, 3, P, 48, 6, c0, c1, log=None,
                             restart=M)
    held = W.generate_pairs(ctx, NX, NY, ELL, ALPHA, _kappa, [7], (1,), 30, 3, P, 48, 6, c0, c1, seed=1,
                            log=None, restart=M)
    cnn, hist = W.train_network(ctx, train, 400, 32, 2e-3, 3, c0, c1, log=None)
    held_loss = W.eval_loss(ctx, cnn, held, 3, batch=32)
    res = W.compare_solves(ctx, cnn, NX, NY, ELL, ALPHA, _kappa(7), 7, P, restart=M)
    print(json.dumps({"first_loss": float(np.mean(hist[:10])), "final_loss": float(np.mean(hist[-50:])),
                      "held_out_loss": held_loss, **res}))
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
