"""Pins of the warm-start network oracle (parity unpinned by the paper, which has no
learned component): forward against an independent correlation routine, the
hand-written backward against central finite differences, Adam's closed-form first
step, and a linear special case."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 7, 6, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    out = cnn.conv3x3(X, W)
    ref = np.zeros_like(out)
    for b in range(2):
        for o in range(4):
            for c in range(3):
                ref[b, :, :, o] += ndimage.correlate(X[b, :, :, c], W[:, :, c, o], mode="constant", cval=0.0)
    assert np.max(np.abs(out - ref)) < 1e-12


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = cnn.init_params(3)
    for k in params:
        params[k] = params[k] + 0.05 * rng.standard_normal(params[k].shape)  # biases non-zero too
    X = rng.standard_normal((2, 6, 5, cnn.C_IN))
    T = rng.standard_normal((2, 6, 5, cnn.C_OUT))
    mask = cnn.border_mask(6, 5, 1)
    L, g = cnn.loss_and_grads(params, X, T, mask)
    h = 1e-6
    for k in ["W1", "b1", "W2", "b2", "W3", "b3"]:
        flat = params[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            Lp = cnn.loss(cnn.forward(params, X)[0], T, mask)
            flat[i] = old - h
            Lm = cnn.loss(cnn.forward(params, X)[0], T, mask)
            flat[i] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, g[k].reshape(-1)[i])


def test_input_gradient_is_adjoint_of_conv():
    """<conv(X, W), D> = <X, conv_grad_input(D, W)> for all X, D."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((1, 5, 8, 4))
    D = rng.standard_normal((1, 5, 8, 3))
    W = rng.standard_normal((3, 3, 4, 3))
    lhs = np.sum(cnn.conv3x3(X, W) * D)
    rhs = np.sum(X * cnn.conv3x3_grad_input(D, W))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_adam_first_step_closed_form():
    opt = cnn.Adam(lr=0.01)
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    p = opt.step(p, g)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> w -= lr * g / (|g| + eps)
    expect = np.array([1.0, -2.0, 3.0]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], expect, rtol=0, atol=1e-15)


def test_linear_special_case():
    """With a single active channel, positive weights and positive inputs the ReLUs are
    inactive and the network is the composition of three correlations (a 7x7 filter)."""
    rng = np.random.default_rng(4)
    params = {k: np.zeros_like(v) for k, v in cnn.init_params(0).items()}
    k1 = rng.uniform(0.1, 1, (3, 3))
    k2 = rng.uniform(0.1, 1, (3, 3))
    k3 = rng.uniform(0.1, 1, (3, 3))
    params["W1"][:, :, 0, 0] = k1
    params["W2"][:, :, 0, 0] = k2
    params["W3"][:, :, 0, 0] = k3
    X = np.zeros((1, 12, 11, cnn.C_IN))
    X[0, :, :, 0] = rng.uniform(0.1, 1, (12, 11))
    Y, _ = cnn.forward(params, X)
    ref = X[0, :, :, 0]
    for k in (k1, k2, k3):
        ref = ndimage.correlate(ref, k, mode="constant", cval=0.0)
    assert np.max(np.abs(Y[0, :, :, 0] - ref)) < 1e-12
    assert np.max(np.abs(Y[0, :, :, 1])) == 0.0
