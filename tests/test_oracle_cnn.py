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


def _res_case(seed=5, Bn=2, H=7, Wd=6):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((Bn, H, Wd, 2))
    R = rng.standard_normal((Bn, H, Wd, 2))
    kap = rng.uniform(0.5, 3.0, (Bn, H, Wd))
    lam = rng.standard_normal(Bn) + 1j * rng.standard_normal(Bn)
    return rng, Y, R, kap, lam


def test_shifted_apply_interior_by_loops():
    """Interior points of the crop operator by the five-point formula written out:
    (B y)_i = (1 - lambda) y_i + sum_faces (kappa_i + kappa_nb)/2 (y_i - y_nb)."""
    _, Y, _, kap, lam = _res_case()
    got = cnn.shifted_apply(Y, kap, lam)
    y = Y[..., 0] + 1j * Y[..., 1]
    for b in range(Y.shape[0]):
        for i in range(1, Y.shape[1] - 1):
            for j in range(1, Y.shape[2] - 1):
                v = (1 - lam[b]) * y[b, i, j]
                for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    kf = 0.5 * (kap[b, i, j] + kap[b, i + di, j + dj])
                    v += kf * (y[b, i, j] - y[b, i + di, j + dj])
                assert abs(got[b, i, j] - v) < 1e-12 * max(1.0, abs(v))


def test_residual_loss_vanishes_at_the_crop_solution():
    """y = (A_crop - lambda I)^{-1} rhat (sparse direct solve) has zero residual."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle.operators import build_A
    _, _, R, kap, lam = _res_case(6)
    Bn, H, Wd, _ = R.shape
    Y = np.empty_like(R)
    for b in range(Bn):
        M = (build_A(2, Wd, H, kap[b].reshape(-1)) - lam[b] * sp.identity(H * Wd)).tocsc()
        y = spla.spsolve(M, (R[b, ..., 0] + 1j * R[b, ..., 1]).reshape(-1)).reshape(H, Wd)
        Y[b, ..., 0], Y[b, ..., 1] = y.real, y.imag
    assert cnn.residual_loss(Y, R, kap, lam, cnn.border_mask(H, Wd, 1)) < 1e-24
    assert cnn.residual_loss(np.zeros_like(R), R, kap, lam, cnn.border_mask(H, Wd, 1)) == pytest.approx(1.0)


def test_residual_loss_without_diffusion():
    """kappa = 0: B = (1 - lambda) I and the loss is a pointwise closed form."""
    _, Y, R, kap, lam = _res_case(7)
    mask = cnn.border_mask(Y.shape[1], Y.shape[2], 1)
    y = Y[..., 0] + 1j * Y[..., 1]
    r = R[..., 0] + 1j * R[..., 1]
    num = np.sum(mask * np.abs(r - (1 - lam[:, None, None]) * y) ** 2, axis=(1, 2))
    den = np.sum(mask * np.abs(r) ** 2, axis=(1, 2))
    assert cnn.residual_loss(Y, R, 0 * kap, lam, mask) == pytest.approx(np.mean(num / den), rel=1e-13)


def test_residual_loss_gradient_matches_finite_differences():
    rng, Y, R, kap, lam = _res_case(8)
    mask = cnn.border_mask(Y.shape[1], Y.shape[2], 1)
    g = cnn.residual_loss_grad(Y, R, kap, lam, mask)
    h = 1e-6
    for idx in [tuple(rng.integers(0, s) for s in Y.shape) for _ in range(12)] + [(0, 0, 0, 1), (1, 3, 2, 0)]:
        Yp, Ym = Y.copy(), Y.copy()
        Yp[idx] += h
        Ym[idx] -= h
        fd = (cnn.residual_loss(Yp, R, kap, lam, mask) - cnn.residual_loss(Ym, R, kap, lam, mask)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_residual_loss_network_gradients_match_finite_differences():
    rng = np.random.default_rng(9)
    params = cnn.init_params(4)
    for k in params:
        params[k] = params[k] + 0.05 * rng.standard_normal(params[k].shape)
    X = rng.standard_normal((2, 6, 5, cnn.C_IN))
    R = rng.standard_normal((2, 6, 5, 2))
    kap = rng.uniform(0.5, 2.0, (2, 6, 5))
    lam = np.array([0.3 - 0.2j, -0.5 + 0.1j])
    mask = cnn.border_mask(6, 5, 1)
    L, g = cnn.residual_loss_and_grads(params, X, R, kap, lam, mask)
    h = 1e-6
    for k in ["W1", "b1", "W2", "b3", "W3"]:
        flat = params[k].reshape(-1)
        for i in rng.choice(flat.size, size=min(5, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + h
            Lp = cnn.residual_loss(cnn.forward(params, X)[0], R, kap, lam, mask)
            flat[i] = old - h
            Lm = cnn.residual_loss(cnn.forward(params, X)[0], R, kap, lam, mask)
            flat[i] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (k, i)


def test_make_inputs_hand_computed_planes():
    """The five input planes of one shift on a 2 x 3 grid, written out by hand: channel
    0/1 the real/imaginary part of rhat divided by the scale, 2/3 the real/imaginary part
    of the shift (constant planes), 4 the normalised log-coefficient (ln kappa - c0)/c1.
    A swapped channel, a missing scale or a wrong normalisation fails it."""
    rhat = np.array([[2.0 + 4.0j, -6.0 + 0.0j, 0.0 + 1.0j],
                     [1.0 - 2.0j, 0.0 + 0.0j, -3.0 - 3.0j]])
    kappa = np.exp(np.array([1.0, 3.0, 5.0, 0.0, 2.0, 7.0]))  # ln kappa = 1, 3, 5, 0, 2, 7
    X = cnn.make_inputs(rhat, 0.25 - 0.5j, kappa, c0=1.0, c1=2.0, scale=2.0)
    assert X.shape == (2, 3, 5)
    expect = {
        0: [[1.0, -3.0, 0.0], [0.5, 0.0, -1.5]],
        1: [[2.0, 0.0, 0.5], [-1.0, 0.0, -1.5]],
        2: [[0.25] * 3, [0.25] * 3],
        3: [[-0.5] * 3, [-0.5] * 3],
        4: [[0.0, 1.0, 2.0], [-0.5, 0.5, 3.0]],
    }
    for c, plane in expect.items():
        assert np.allclose(X[..., c], plane, rtol=0, atol=1e-15), c
