"""GPU parity of the warm-start network kernels against the float64 oracle, and the
warm-started solve.

The oracle runs on the same bf16-representable inputs and bf16-rounded weights the
matrix cores see; the remaining differences come from bf16 rounding (unit roundoff
u = 2^-8 = 3.9e-3) of the two hidden activations (forward: bound 1e-2 ~ 2.5 u) and, for
the gradients, of the tensors on each parameter's path plus ReLU decisions on
pre-activations within u of zero.  The bounds grow with the path: the last layer's
gradient sees one rounded activation (bound 1e-2 ~ 2.5 u; measured <= 1.3e-3), the
middle layer's also a back-propagated gradient and the first activation (3e-2 ~ 8 u;
measured <= 1.5e-2), the first layer's up to five rounded tensors (5e-2 ~ 13 u;
measured <= 3.8e-2).
"""


import numpy as np
import pytest
import torch

from oracle import cnn as ocnn
from oracle import operators as ops
from oracle.precision import to_bfloat16
from paper_2506_03947_amd import api
from synth import first_block_rhs, lognormal_kappa
from tests import gpu_util as G

L = api.L
pytestmark = pytest.mark.gpu

# relative gradient bound per parameter tensor (see the module docstring)
GRAD_TOL = {"W1": 5e-2, "b1": 5e-2, "W2": 3e-2, "b2": 3e-2, "W3": 1e-2, "b3": 1e-2}


def packed_from_oracle(params):
    """Oracle dict -> packed parameter vector [W [t][out][in] (9x16x16), b (16)] x 3."""
    out = []
    for k in ("1", "2", "3"):
        W = params["W" + k]
        P = np.zeros((3, 3, 16, 16))
        P[:, :, : W.shape[3], : W.shape[2]] = np.transpose(W, (0, 1, 3, 2))
        b = np.zeros(16)
        b[: params["b" + k].size] = params["b" + k]
        out += [P.reshape(-1), b]
    return np.concatenate(out)


def oracle_from_packed(vec):
    p = {}
    sizes = {"1": (5, 16), "2": (16, 16), "3": (16, 2)}
    o = 0
    for k in ("1", "2", "3"):
        P = vec[o:o + 2304].reshape(3, 3, 16, 16)
        cin, cout = sizes[k]
        p["W" + k] = np.transpose(P, (0, 1, 3, 2))[:, :, :cin, :cout].astype(np.float64)
        p["b" + k] = vec[o + 2304:o + 2304 + cout].astype(np.float64)
        o += 2320
    return p


def bf16_bits(x):
    """bf16-representable float array -> uint16 bit patterns as int16 tensor."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32) >> 16
    return torch.from_numpy(u.astype(np.uint16).view(np.int16)).to("cuda:0")


def _setup(seed=0, B=3, H=20, W=37):
    rng = np.random.default_rng(seed)
    params = ocnn.init_params(seed)
    for k in params:
        if k.startswith("b"):
            params[k] = 0.1 * rng.standard_normal(params[k].shape)
    vec = packed_from_oracle(params).astype(np.float32)
    qparams = oracle_from_packed(vec)  # float32 master values
    for k in qparams:
        if k.startswith("W"):
            qparams[k] = to_bfloat16(qparams[k])  # what the matrix cores multiply with
    X = np.zeros((B, H, W, 16))
    X[..., :5] = to_bfloat16(rng.standard_normal((B, H, W, 5)))
    return rng, vec, qparams, X


def test_forward_parity():
    rng, vec, qp, X = _setup()
    B, H, W = X.shape[:3]
    cnn = api.ac_cnn_create(G.ctx())
    api.ac_cnn_set_params(cnn, vec, 0.0, 1.0)
    ws = api.workspace(api.ac_cnn_workspace_size(B, H, W))
    y = torch.zeros(B * H * W * 2, dtype=torch.float32, device="cuda:0")
    api.ac_cnn_forward(cnn, bf16_bits(X), B, H, W, y, ws)
    ref, _ = ocnn.forward(qp, X[..., :5])
    got = G.host(y).reshape(B, H, W, 2)
    assert G.rel(got, ref) < 1e-2


def test_gradient_parity_and_loss():
    rng, vec, qp, X = _setup(1, B=2, H=24, W=40)
    B, H, W = X.shape[:3]
    T = rng.standard_normal((B, H, W, 2))
    border = 2
    mask = ocnn.border_mask(H, W, border)
    tnorm = np.sum(mask[None, :, :, None] * T ** 2, axis=(1, 2, 3))
    cnn = api.ac_cnn_create(G.ctx())
    api.ac_cnn_set_params(cnn, vec, 0.0, 1.0)
    ws = api.workspace(api.ac_cnn_workspace_size(B, H, W))
    loss, g = api.ac_cnn_grad(cnn, bf16_bits(X), G.dev(T.astype(np.float32)),
                              G.dev(tnorm.astype(np.float32)), border, B, H, W, ws, want_grad=True)
    L_ref, g_ref = ocnn.loss_and_grads(qp, X[..., :5], T, mask)
    assert abs(loss - L_ref) < 1e-2 * L_ref
    got = oracle_from_packed(g)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert G.rel(got[k], g_ref[k]) < GRAD_TOL[k], k
    # parameters outside the network get no gradient
    assert np.all(g[0:2304].reshape(9, 16, 16)[:, :, 5:] == 0)
    assert np.all(g[2 * 2320:2 * 2320 + 2304].reshape(9, 16, 16)[:, 2:, :] == 0)


def test_residual_loss_gradient_parity():
    """Residual-space loss of the crop's shifted operator: loss and every parameter
    gradient against the oracle (same bf16 error budget as the solution-space loss)."""
    rng, vec, qp, X = _setup(3, B=3, H=24, W=40)
    B, H, W = X.shape[:3]
    R = rng.standard_normal((B, H, W, 2)).astype(np.float32).astype(np.float64)
    kap = rng.uniform(0.5, 4.0, (B, H, W)).astype(np.float32).astype(np.float64)
    lam = (rng.uniform(-0.6, 0.6, B) + 1j * rng.uniform(-0.6, 0.6, B)).astype(np.complex64).astype(np.complex128)
    border = 2
    mask = ocnn.border_mask(H, W, border)
    rnorm = np.sum(mask[None] * (R[..., 0] ** 2 + R[..., 1] ** 2), axis=(1, 2))
    cnn = api.ac_cnn_create(G.ctx())
    api.ac_cnn_set_params(cnn, vec, 0.0, 1.0)
    ws = api.workspace(api.ac_cnn_workspace_size(B, H, W))
    lam2 = np.stack([lam.real, lam.imag], -1).astype(np.float32)
    loss, g = api.ac_cnn_grad_residual(cnn, bf16_bits(X), G.dev(R.astype(np.float32)), G.dev(kap.astype(np.float32)),
                                       G.dev(lam2), G.dev(rnorm.astype(np.float32)), border, B, H, W, ws,
                                       want_grad=True)
    L_ref, g_ref = ocnn.residual_loss_and_grads(qp, X[..., :5], R, kap, lam, mask)
    assert abs(loss - L_ref) < 1e-2 * L_ref
    got = oracle_from_packed(g)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert G.rel(got[k], g_ref[k]) < GRAD_TOL[k], k


def test_residual_loss_rejects_zero_border():
    B, H, W = 1, 8, 8
    cnn = api.ac_cnn_create(G.ctx())
    ws = api.workspace(api.ac_cnn_workspace_size(B, H, W))
    z = torch.zeros(B * H * W * 16, dtype=torch.int16, device="cuda:0")
    f = torch.ones(B * H * W * 2, dtype=torch.float32, device="cuda:0")
    with pytest.raises(api.L.AlphacircError):
        api.ac_cnn_grad_residual(cnn, z, f, f[: B * H * W], f[:2], f[:1], 0, B, H, W, ws)


def test_adam_step_matches_oracle():
    rng, vec, qp, X = _setup(2, B=2, H=16, W=32)
    B, H, W = X.shape[:3]
    T = rng.standard_normal((B, H, W, 2))
    mask = ocnn.border_mask(H, W, 1)
    tnorm = np.sum(mask[None, :, :, None] * T ** 2, axis=(1, 2, 3))
    cnn = api.ac_cnn_create(G.ctx())
    api.ac_cnn_set_params(cnn, vec, 0.0, 1.0)
    ws = api.workspace(api.ac_cnn_workspace_size(B, H, W))
    api.ac_cnn_grad(cnn, bf16_bits(X), G.dev(T.astype(np.float32)), G.dev(tnorm.astype(np.float32)), 1, B, H, W, ws)
    lr = 1e-3
    api.ac_cnn_adam_step(cnn, lr)
    new, _, _ = api.ac_cnn_get_params(cnn)
    # oracle: its own gradient and Adam from the same starting point
    start = oracle_from_packed(vec)
    _, g_ref = ocnn.loss_and_grads(qp, X[..., :5], T, mask)
    opt = ocnn.Adam(lr=lr)
    ref = opt.step({k: v.copy() for k, v in start.items()}, g_ref)
    got = oracle_from_packed(new)
    for k in ref:
        step_ref = ref[k] - start[k]
        step_got = got[k] - start[k]
        # first Adam step is lr * g / (|g| + eps): +-lr wherever the gradient is not tiny
        big = np.abs(g_ref[k]) > 1e-3 * np.max(np.abs(g_ref[k]))
        assert np.all(np.abs(step_got - step_ref) <= 2.1 * lr)
        assert np.mean(np.sign(step_got[big]) == np.sign(step_ref[big])) > 0.97, k


def _solve_problem():
    nx, ny, ell, alpha = 96, 64, 6, 1e-2
    kap = lognormal_kappa(nx, ny, 20.0, 5.0, 1.0, seed=5)
    A = ops.build_A(2, nx, ny, kap)
    b = first_block_rhs(nx * ny, ell, seed=0)
    p = G.problem(2, nx, ny, kap, ell, alpha)
    return p, A, b, kap, ell


@pytest.mark.parametrize("scale", [1.0, 1e4])
def test_warm_started_solve_and_fallback(scale):
    """A random network (scale 1) and a corrupted one (scale 1e4: every guess rejected):
    the warm-started FGMRES solve still converges to the sequential solution."""
    p, A, b, kap, ell = _solve_problem()
    params = ocnn.init_params(7)
    vec = (packed_from_oracle(params) * scale).astype(np.float32)
    cnn = api.ac_cnn_create(G.ctx())
    lk = np.log(kap)
    api.ac_cnn_set_params(cnn, vec, float(lk.mean()), float(lk.std()))
    api.ac_cnn_set_guess_policy(cnn, False, 1.0)
    api.ac_problem_attach_cnn(p, cnn)
    opts = api.Opts(precision=L.AC_PREC_MIXED_BF16K, inner=L.AC_INNER_CHEB_CNN, p=8, tol=1e-10, restart_m=20,
                    max_outer=500)
    ws = api.workspace(api.ac_solve_workspace_size(p, opts))
    x = G.dev(np.zeros_like(b))
    info = api.ac_solve(p, opts, G.dev(b), x, ws)
    assert info["converged"], info
    assert G.rel(G.host(x), ops.sequential_solve(A, b, ell)) < 1e-6
    if scale > 1:
        assert info["cnn_fallbacks"] == info["outer_iters"] * p.ns


def test_cnn_inputs_layout():
    """Network inputs for each shift slot: scaled real/imaginary parts of rhat, the
    shift, and the normalised ln kappa (checked against the oracle's make_inputs)."""
    from oracle import precond as pc
    p, A, b, kap, ell = _solve_problem()
    cnn = api.ac_cnn_create(G.ctx())
    api.ac_cnn_set_params(cnn, np.zeros(api.ac_cnn_param_count(), np.float32), 3.0, 1.5)
    r = np.random.default_rng(3).standard_normal(ell * p.n)
    off = api.ac_spectral_offsets(p, 0)
    rhat = torch.zeros(off[-1], dtype=torch.float64, device="cuda:0")
    api.ac_tdft_forward(p, 0, G.dev(r), rhat)
    x = torch.zeros(p.ns * p.n * 16, dtype=torch.int16, device="cuda:0")
    rs = torch.zeros((p.ns, p.n, 2), dtype=torch.float32, device="cuda:0")
    scales = api.ac_cnn_make_inputs(p, cnn, 0, rhat, x, rs)
    bits = G.host(x).view(np.uint16).astype(np.uint32) << 16
    got = bits.view(np.float32).reshape(p.ns, 64, 96, 16)
    got_rs = G.host(rs).reshape(p.ns, 64, 96, 2)
    R = pc.forward_transform(r, ell, 1e-2)
    lam = pc.shifts(ell, 1e-2)
    for s, m in enumerate(api.slot_order(p)):
        sc = np.sqrt(np.mean(np.abs(R[m]) ** 2))
        assert abs(scales[s] - sc) < 1e-12 * sc
        ref = ocnn.make_inputs(R[m].reshape(64, 96), lam[m], kap, 3.0, 1.5, sc)
        assert G.max_rel(got[s, :, :, :5], to_bfloat16(ref)) < 1e-2
        assert not got[s, :, :, 5:].any()
        # the float32 scaled right-hand side: channels 0 and 1 of the oracle's planes
        assert G.max_rel(got_rs[s], ref[..., :2]) < 1e-6


@pytest.mark.parametrize("precision", [L.AC_PREC_FP64, L.AC_PREC_MIXED_BF16K])
@pytest.mark.parametrize("scaling", [False, True])
def test_fused_inference_equals_layer_by_layer(precision, scaling):
    """The fused kernel (all layers per 16 x 16 tile in LDS) against input packing +
    three convolution launches + output scaling, on a grid ragged against the tiles:
    identical guesses without the minimal-residual factor (same roundings, same tap
    order), equal to float32 rounding with it."""
    nx, ny, ell = 100, 70, 6
    rng = np.random.default_rng(11)
    kap = 20.0 * (1.0 + 0.05 * rng.uniform(-1, 1, nx * ny))  # nearly constant: the hand-made guess is kept
    p = G.problem(2, nx, ny, kap, ell, 1e-2)
    # a network whose guesses are kept: x0 ~ rhat / (1 + 4 mean kappa) through
    # sign-split ReLU channels (centre taps), plus small perturbations of every weight
    w = 1.0 / (1.0 + 4.0 * float(np.mean(kap)))
    params = {k: 0.01 * rng.standard_normal(v.shape) for k, v in ocnn.init_params(12).items()}
    params["W3"] *= w
    for cin, cout, sgn in ((0, 0, 1.0), (0, 1, -1.0), (1, 2, 1.0), (1, 3, -1.0)):
        params["W1"][1, 1, cin, cout] += sgn
    for k in range(4):
        params["W2"][1, 1, k, k] += 1.0
    for cin, cout, sgn in ((0, 0, 1.0), (1, 0, -1.0), (2, 1, 1.0), (3, 1, -1.0)):
        params["W3"][1, 1, cin, cout] += sgn * w
    cnn = api.ac_cnn_create(G.ctx())
    api.ac_cnn_set_params(cnn, packed_from_oracle(params).astype(np.float32), float(np.log(kap).mean()), 1.0)
    api.ac_cnn_set_guess_policy(cnn, scaling, 1.0)
    api.ac_problem_attach_cnn(p, cnn)
    off = api.ac_spectral_offsets(p, precision)
    dt = torch.float64 if precision == L.AC_PREC_FP64 else torch.float32
    rhat = torch.zeros(off[-1], dtype=dt, device="cuda:0")
    api.ac_tdft_forward(p, precision, G.dev(rng.standard_normal(ell * nx * ny)), rhat)
    ws = api.workspace(api.ac_cnn_guess_workspace_size(p))
    out = []
    for fused in (False, True):
        api.ac_cnn_set_inference(cnn, fused)
        x0 = torch.zeros_like(rhat)
        rej = api.ac_cnn_guess(p, precision, rhat, x0, ws)
        out.append((G.host(x0), rej))
    assert out[0][1] == out[1][1] < p.ns
    if scaling:
        assert G.max_rel(out[1][0], out[0][0]) < 1e-5
    else:
        assert np.array_equal(out[1][0], out[0][0])
    assert np.abs(out[1][0]).max() > 0
