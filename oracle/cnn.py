"""Learned warm start for the shifted inner solves: oracle side (float64, numpy).

The network is not part of the paper; it is the learned initial guess for the
inner Chebyshev solves of Section 3 (the Chebyshev steps then correct it).  Three
3x3 convolutions with zero padding, 5 -> 16 -> 16 -> 2 channels, ReLU after the
first two:

  inputs (per shift m and grid point): Re rhat_m / s_m, Im rhat_m / s_m,
  Re lambda_m, Im lambda_m, (ln kappa - c0) / c1;  s_m = RMS(rhat_m);
  outputs: Re x0_m / s_m, Im x0_m / s_m.

Convolution is cross-correlation: conv(X, W)[y, x, o] =
sum_{dy, dx in -1..1} sum_c X[y+dy, x+dx, c] W[dy+1, dx+1, c, o] (+ bias).
Two losses over a batch of crops with a border mask M (zero within `border`
cells of a crop edge):
  solution space:  L = (1/B) sum_b sum M |Y_b - T_b|^2 / sum M |T_b|^2;
  residual space:  L = (1/B) sum_b sum M |rhat_b - B_b y_b|^2 / sum M |rhat_b|^2,
where y_b = Y_b[..., 0] + i Y_b[..., 1] and B_b = A_b - lambda_b I is the shifted
operator of Section 3 restricted to the crop (A_b from the coefficient crop, zero
outside it).  The residual loss is what the warm start must make small: the
Chebyshev steps that follow contract the initial residual, and the guess is
rejected when its residual is not below that of x0 = 0.
Optimiser: Adam (Kingma & Ba 2015) with bias correction.

Parity unpinned by the paper (it has no learned component).  Pinned here by
finite differences of the hand-written backward pass, by an independent
correlation routine (scipy.ndimage.correlate) for the forward pass, and by the
closed-form first Adam step.
"""

from __future__ import annotations

import numpy as np

from .operators import build_A

C_IN, C_HID, C_OUT = 5, 16, 2


def init_params(seed: int = 0):
    """He-normal initialisation, zero biases."""
    rng = np.random.default_rng(seed)

    def he(cin, cout):
        return rng.standard_normal((3, 3, cin, cout)) * np.sqrt(2.0 / (9 * cin))

    return {"W1": he(C_IN, C_HID), "b1": np.zeros(C_HID),
            "W2": he(C_HID, C_HID), "b2": np.zeros(C_HID),
            "W3": he(C_HID, C_OUT) * 0.1, "b3": np.zeros(C_OUT)}


def conv3x3(X: np.ndarray, W: np.ndarray, b=None) -> np.ndarray:
    """X: (B, H, Wd, Cin), W: (3, 3, Cin, Cout) -> (B, H, Wd, Cout), zero padding."""
    B, H, Wd, _ = X.shape
    Xp = np.pad(X, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((B, H, Wd, W.shape[3]))
    for ky in range(3):
        for kx in range(3):
            out += Xp[:, ky:ky + H, kx:kx + Wd, :] @ W[ky, kx]
    if b is not None:
        out += b
    return out


def forward(params, X):
    """Returns the output and the cache needed by backward."""
    Z1 = conv3x3(X, params["W1"], params["b1"])
    A1 = np.maximum(Z1, 0.0)
    Z2 = conv3x3(A1, params["W2"], params["b2"])
    A2 = np.maximum(Z2, 0.0)
    Y = conv3x3(A2, params["W3"], params["b3"])
    return Y, (X, Z1, A1, Z2, A2)


def border_mask(H: int, Wd: int, border: int) -> np.ndarray:
    m = np.zeros((H, Wd))
    m[border:H - border, border:Wd - border] = 1.0
    return m


def loss(Y, T, mask):
    """Mean over the batch of the masked relative squared error."""
    M = mask[None, :, :, None]
    num = np.sum(M * (Y - T) ** 2, axis=(1, 2, 3))
    den = np.sum(M * T ** 2, axis=(1, 2, 3))
    return float(np.mean(num / den))


def loss_grad(Y, T, mask):
    M = mask[None, :, :, None]
    den = np.sum(M * T ** 2, axis=(1, 2, 3))
    return 2.0 * M * (Y - T) / (Y.shape[0] * den[:, None, None, None])


def conv3x3_grad_input(dOut, W):
    """d/dX of conv3x3: dX[y, x, c] = sum_{ky,kx,o} dOut[y - ky + 1, x - kx + 1, o] W[ky, kx, c, o]."""
    B, H, Wd, _ = dOut.shape
    dp = np.pad(dOut, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dX = np.zeros((B, H, Wd, W.shape[2]))
    for ky in range(3):
        for kx in range(3):
            # output pixel (y', x') = (y - ky + 1, x - kx + 1) used input (y, x) with tap (ky, kx)
            dX += dp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + Wd, :] @ W[ky, kx].T
    return dX


def conv3x3_grad_weight(X, dOut):
    """dW[ky, kx, c, o] = sum_{b, y, x} X[b, y + ky - 1, x + kx - 1, c] dOut[b, y, x, o]."""
    B, H, Wd, _ = X.shape
    Xp = np.pad(X, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dW = np.zeros((3, 3, X.shape[3], dOut.shape[3]))
    for ky in range(3):
        for kx in range(3):
            patch = Xp[:, ky:ky + H, kx:kx + Wd, :].reshape(-1, X.shape[3])
            dW[ky, kx] = patch.T @ dOut.reshape(-1, dOut.shape[3])
    return dW


def backward(params, cache, dY):
    X, Z1, A1, Z2, A2 = cache
    g = {}
    g["W3"] = conv3x3_grad_weight(A2, dY)
    g["b3"] = dY.sum(axis=(0, 1, 2))
    dZ2 = conv3x3_grad_input(dY, params["W3"]) * (Z2 > 0)
    g["W2"] = conv3x3_grad_weight(A1, dZ2)
    g["b2"] = dZ2.sum(axis=(0, 1, 2))
    dZ1 = conv3x3_grad_input(dZ2, params["W2"]) * (Z1 > 0)
    g["W1"] = conv3x3_grad_weight(X, dZ1)
    g["b1"] = dZ1.sum(axis=(0, 1, 2))
    return g


def loss_and_grads(params, X, T, mask):
    Y, cache = forward(params, X)
    L = loss(Y, T, mask)
    return L, backward(params, cache, loss_grad(Y, T, mask))


def shifted_apply(Y, kappa, lam):
    """(A_b - lambda_b I) y_b for every crop b: Y (B, H, W, 2) real/imaginary parts,
    kappa (B, H, W), lam (B,) complex; A_b is the operator of the crop with zero
    Dirichlet values outside it.  Returns a complex (B, H, W) array."""
    Bn, H, Wd, _ = Y.shape
    out = np.empty((Bn, H, Wd), dtype=np.complex128)
    for b in range(Bn):
        A = build_A(2, Wd, H, kappa[b].reshape(-1))
        y = (Y[b, ..., 0] + 1j * Y[b, ..., 1]).reshape(-1)
        out[b] = (A @ y - lam[b] * y).reshape(H, Wd)
    return out


def residual_loss(Y, Rhat, kappa, lam, mask):
    """Mean over the batch of the masked relative squared residual."""
    r = Rhat[..., 0] + 1j * Rhat[..., 1]
    e = mask[None] * (r - shifted_apply(Y, kappa, lam))
    num = np.sum(np.abs(e) ** 2, axis=(1, 2))
    den = np.sum(mask[None] * np.abs(r) ** 2, axis=(1, 2))
    return float(np.mean(num / den))


def residual_loss_grad(Y, Rhat, kappa, lam, mask):
    """dL/dY: with e = M (rhat - B y), the gradient with respect to (Re y, Im y) is
    -2 B^H M e / (batch * den); B^H = A - conj(lambda) I since A is symmetric."""
    Bn = Y.shape[0]
    r = Rhat[..., 0] + 1j * Rhat[..., 1]
    e = mask[None] * (r - shifted_apply(Y, kappa, lam))
    den = np.sum(mask[None] * np.abs(r) ** 2, axis=(1, 2))
    E = np.stack([e.real, e.imag], axis=-1)
    g = -2.0 * shifted_apply(E, kappa, np.conj(lam)) / (Bn * den[:, None, None])
    return np.stack([g.real, g.imag], axis=-1)


def residual_loss_and_grads(params, X, Rhat, kappa, lam, mask):
    Y, cache = forward(params, X)
    return residual_loss(Y, Rhat, kappa, lam, mask), backward(
        params, cache, residual_loss_grad(Y, Rhat, kappa, lam, mask))


class Adam:
    """Adam with bias correction; state per parameter name."""

    def __init__(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m, self.v = {}, {}

    def step(self, params, grads):
        self.t += 1
        for k, g in grads.items():
            m = self.m.get(k, np.zeros_like(g))
            v = self.v.get(k, np.zeros_like(g))
            m = self.b1 * m + (1 - self.b1) * g
            v = self.b2 * v + (1 - self.b2) * g * g
            self.m[k], self.v[k] = m, v
            mh = m / (1 - self.b1 ** self.t)
            vh = v / (1 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return params


def make_inputs(rhat_m: np.ndarray, lam_m: complex, kappa: np.ndarray, c0: float, c1: float, scale: float):
    """Network input planes (H, W, 5) for one shift from its transformed residual
    (complex (H, W)), its shift and the coefficient field."""
    H, Wd = rhat_m.shape
    X = np.empty((H, Wd, C_IN))
    X[..., 0] = rhat_m.real / scale
    X[..., 1] = rhat_m.imag / scale
    X[..., 2] = lam_m.real
    X[..., 3] = lam_m.imag
    X[..., 4] = (np.log(kappa.reshape(H, Wd)) - c0) / c1
    return X
