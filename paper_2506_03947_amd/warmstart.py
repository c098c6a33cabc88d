"""Training and evaluation of the learned warm start, driven through the C ABI.

Pairs come from the method itself: for a problem (grid, kappa, l, alpha) and a
right-hand side, plain nested-Chebyshev FGMRES records the vectors it hands to the
preconditioner (its Arnoldi basis vectors); each is an input the warm start will
meet.  Its scaled time-DFT gives, for every solved shift m, the network
input planes and the field rhat_m / s_m.  Random crops of these (with the matching
coefficient crop and the shift) form the training set.  The loss is the relative
residual of the guess under the shifted operator of the crop, which is the quantity
the inner Chebyshev steps contract and the fallback test checks; training runs the
library's forward, residual-loss, backward and Adam kernels.

Checkpoints are JSON: the parameter vector, the ln-kappa normalisation and the
training record.  The coefficient fields and right-hand sides come from the caller
(callables returning host arrays); `bench.py --mode warmstart` runs the whole
generate / train / compare sequence on the 1024 x 1024 workload.
"""

from __future__ import annotations

import json
import math
import time

import numpy as np
import torch

from . import api

L = api.L
PAIR_PREC = L.AC_PREC_MIXED_FP32K


def make_problem(ctx, nx, ny, ell, alpha, kappa):
    return api.ac_problem_create(ctx, 2, nx, ny, torch.as_tensor(kappa, device="cuda:0"), ell, alpha)


class _Buffers:
    def __init__(self):
        self.ws = {}

    def get(self, key, nbytes):
        if key not in self.ws or self.ws[key].numel() < nbytes:
            self.ws[key] = api.workspace(nbytes)
        return self.ws[key]


def preconditioner_inputs(prob, b, p_inner, count, bufs, restart=8, warm=False):
    """The first `count` vectors FGMRES(restart) from x = 0 hands to the preconditioner
    (its Arnoldi basis vectors), recorded by the library; with warm=True the solve uses
    the attached network, so the inputs carry that network's own residual patterns."""
    inner = L.AC_INNER_CHEB_CNN if warm else L.AC_INNER_CHEB
    opts = api.Opts(precision=L.AC_PREC_MIXED_BF16K, inner=inner, p=p_inner, tol=1e-300, restart_m=restart,
                    max_outer=count)
    rec = torch.empty((count, prob.ell * prob.n), dtype=torch.float64, device="cuda:0")
    x = torch.zeros(prob.ell * prob.n, dtype=torch.float64, device="cuda:0")
    _, done = api.ac_solve_record(prob, opts, b, x, bufs.get("solve", api.ac_solve_workspace_size(prob, opts)), rec)
    return rec[:done]


def field_pairs(prob, cnn, r):
    """For one block residual r: network inputs [l_s, N, 16] (bf16 bits), the scaled
    transformed residual [l_s, N, 2] (float) and the shifts [l_s, 2], in slot order
    (all formed by the library's transform and input kernels)."""
    off = api.ac_spectral_offsets(prob, PAIR_PREC)
    rhat = torch.zeros(off[-1], dtype=torch.float32, device="cuda:0")
    api.ac_tdft_forward(prob, PAIR_PREC, r, rhat)
    X = torch.zeros(prob.ns * prob.n * 16, dtype=torch.int16, device="cuda:0")
    R = torch.empty((prob.ns, prob.n, 2), dtype=torch.float32, device="cuda:0")
    api.ac_cnn_make_inputs(prob, cnn, PAIR_PREC, rhat, X, R)
    lam_all = api.ac_problem_shifts(prob)
    lam = torch.tensor([[lam_all[m].real, lam_all[m].imag] for m in api.slot_order(prob)], dtype=torch.float32)
    return X.view(prob.ns, -1, 16), R, lam


class PairSet:
    """Crops on the device: inputs X [P, H, W, 16] (bf16 bits), scaled residual R
    [P, H, W, 2], coefficient K [P, H, W], shift LAM [P, 2]."""

    def __init__(self, X, R, K, LAM):
        self.X, self.R, self.K, self.LAM = X, R, K, LAM

    def __len__(self):
        return self.X.shape[0]

    def join(self, other):
        return PairSet(torch.cat([self.X, other.X]), torch.cat([self.R, other.R]), torch.cat([self.K, other.K]),
                       torch.cat([self.LAM, other.LAM]))

    def rnorm(self, border):
        H, W = self.R.shape[1:3]
        return self.R[:, border:H - border, border:W - border].pow(2).sum((1, 2, 3)).contiguous()


def generate_pairs(ctx, nx, ny, ell, alpha, kappa_fn, kappa_seeds, rhs_fn, b_seeds, n_record, pick_every, p_inner,
                   crop, crops_per_plane, c0, c1, seed=0, log=print, net=None, restart=8):
    """Crops from every `pick_every`-th of the first `n_record` preconditioner inputs
    of solves for each coefficient field kappa_fn(seed) and right-hand side
    rhs_fn(seed) (host arrays from the caller's input generators): plain solves, or
    solves warm-started by `net` when given."""
    rng = np.random.default_rng(seed)
    Xs, Rs, Ks, Ls = [], [], [], []
    for ks in kappa_seeds:
        kap = kappa_fn(ks)
        prob = make_problem(ctx, nx, ny, ell, alpha, kap)
        kdev = torch.as_tensor(kap, dtype=torch.float32, device="cuda:0").view(ny, nx)
        cnn = api.ac_cnn_create(ctx)
        api.ac_cnn_set_params(cnn, np.zeros(api.ac_cnn_param_count(), np.float32), c0, c1)
        bufs = _Buffers()
        if net is not None:
            api.ac_problem_attach_cnn(prob, net)
        for bs in b_seeds:
            b = torch.as_tensor(rhs_fn(bs), device="cuda:0")
            inputs = preconditioner_inputs(prob, b, p_inner, n_record, bufs, restart=restart, warm=net is not None)
            for v in inputs[::pick_every]:
                X, R, lam = field_pairs(prob, cnn, v.contiguous())
                X = X.view(prob.ns, ny, nx, 16)
                R = R.view(prob.ns, ny, nx, 2)
                for s in range(prob.ns):
                    for y0, x0 in zip(rng.integers(0, ny - crop + 1, crops_per_plane),
                                      rng.integers(0, nx - crop + 1, crops_per_plane)):
                        Xs.append(X[s, y0:y0 + crop, x0:x0 + crop].clone())
                        Rs.append(R[s, y0:y0 + crop, x0:x0 + crop].clone())
                        Ks.append(kdev[y0:y0 + crop, x0:x0 + crop].clone())
                        Ls.append(lam[s])
            del inputs
        if log:
            log(f"kappa seed {ks}: {len(Xs)} pairs")
        del prob, cnn, bufs
    return PairSet(torch.stack(Xs), torch.stack(Rs), torch.stack(Ks), torch.stack(Ls).to("cuda:0"))


def initial_params(seed, last_scale=0.1):
    """Fan-in uniform initialisation (weights and biases in +-1/sqrt(9 fan_in)), last
    layer scaled down so the first guesses are small: the shifted operator multiplies
    output noise by up to 1 + 8 max(kappa), and a larger start (He-normal) leaves
    the residual loss stuck near the zero-guess value."""
    rng = np.random.default_rng(seed)
    vec = np.zeros(api.ac_cnn_param_count(), dtype=np.float32)
    fan = (5, 16, 16)
    cout = (16, 16, 2)
    for layer in range(3):
        bnd = 1.0 / math.sqrt(9 * fan[layer])
        sc = last_scale if layer == 2 else 1.0
        W = np.zeros((9, 16, 16), dtype=np.float32)
        W[:, : cout[layer], : fan[layer]] = sc * rng.uniform(-bnd, bnd, (9, cout[layer], fan[layer]))
        o = layer * 2320
        vec[o: o + 2304] = W.reshape(-1)
        vec[o + 2304: o + 2304 + cout[layer]] = sc * rng.uniform(-bnd, bnd, cout[layer])
    return vec


def train_network(ctx, pairs, steps, batch, lr, border, c0, c1, seed=0, log=print, log_every=200, cnn=None):
    """Adam with cosine learning-rate decay on random mini-batches of crops, residual
    loss; continues training `cnn` (parameters and optimiser state) when given."""
    if cnn is None:
        cnn = api.ac_cnn_create(ctx)
        api.ac_cnn_set_params(cnn, initial_params(seed), c0, c1)
    H, W = pairs.X.shape[1], pairs.X.shape[2]
    ws = api.workspace(api.ac_cnn_workspace_size(batch, H, W))
    rn = pairs.rnorm(border)
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for it in range(steps):
        idx = torch.randint(0, len(pairs), (batch,), generator=g).to("cuda:0")
        loss, _ = api.ac_cnn_grad_residual(cnn, pairs.X[idx].contiguous(), pairs.R[idx].contiguous(),
                                           pairs.K[idx].contiguous(), pairs.LAM[idx].contiguous(),
                                           rn[idx].contiguous(), border, batch, H, W, ws)
        api.ac_cnn_adam_step(cnn, lr * 0.5 * (1 + math.cos(math.pi * it / steps)))
        hist.append(loss)
        if log and (it % log_every == 0 or it == steps - 1):
            log(f"step {it}: loss {np.mean(hist[-log_every:]):.4f}")
    return cnn, hist


def eval_loss(ctx, cnn, pairs, border, batch=64):
    """Mean residual loss of a network over a pair set (no update)."""
    H, W = pairs.X.shape[1], pairs.X.shape[2]
    ws = api.workspace(api.ac_cnn_workspace_size(batch, H, W))
    rn = pairs.rnorm(border)
    tot, cnt = 0.0, 0
    for i in range(0, len(pairs) - batch + 1, batch):
        sl = slice(i, i + batch)
        loss, _ = api.ac_cnn_grad_residual(cnn, pairs.X[sl].contiguous(), pairs.R[sl].contiguous(),
                                           pairs.K[sl].contiguous(), pairs.LAM[sl].contiguous(),
                                           rn[sl].contiguous(), border, batch, H, W, ws)
        tot += loss * batch
        cnt += batch
    return tot / max(cnt, 1)


def inner_gain(prob, cnn, r, p_inner, bufs):
    """Inner residuals per shift (m = 0..l_s-1) for the transformed residual of r: of the
    network's guess, and after p_inner Chebyshev steps from zero and from the guess."""
    prec = L.AC_PREC_MIXED_BF16K
    off = api.ac_spectral_offsets(prob, prec)
    rhat = torch.zeros(off[-1], dtype=torch.float32, device="cuda:0")
    api.ac_tdft_forward(prob, prec, r, rhat)
    api.ac_problem_attach_cnn(prob, cnn)
    x0 = torch.zeros_like(rhat)
    api.ac_cnn_guess(prob, prec, rhat, x0, bufs.get("guess", api.ac_cnn_guess_workspace_size(prob)))
    opts = api.Opts(precision=prec, p=p_inner)
    ws = bufs.get("prec", api.ac_prec_workspace_size(prob, opts))
    y_cold = torch.zeros_like(rhat)
    y_warm = torch.zeros_like(rhat)
    api.ac_shifted_cheb(prob, opts, rhat, None, y_cold, ws)
    api.ac_shifted_cheb(prob, opts, rhat, x0, y_warm, ws)
    return {"guess": api.ac_shifted_residual(prob, prec, rhat, x0).tolist(),
            "cold": api.ac_shifted_residual(prob, prec, rhat, y_cold).tolist(),
            "warm": api.ac_shifted_residual(prob, prec, rhat, y_warm).tolist()}


def compare_solves(ctx, cnn, nx, ny, ell, alpha, kappa, b, p_inner, tol=1e-8, restart=8, reps=1,
                   modes=("plain", "cnn", "cnn_cycle"), fp64_plain=False):
    """Plain and warm-started FGMRES on one problem (b: host right-hand side): the plain
    method (complex64 + bf16 kappa inner; with fp64_plain also float64 inner), the network
    on every preconditioner input (cnn) and on the first vector of each cycle only
    (cnn_cycle), and as a minimal-residual correction before each cycle (cnn_mr): outer iterations, best wall time of `reps`, fallbacks, the solutions'
    difference to the float64 plain solution when it was run, plus the mean inner residuals per
    shift on inputs the plain method's preconditioner receives; out["x"] holds each
    solution (device tensors)."""
    prob = make_problem(ctx, nx, ny, ell, alpha, kappa)
    api.ac_problem_attach_cnn(prob, cnn)
    bd = torch.as_tensor(b, device="cuda:0")
    out = {}
    bufs = _Buffers()
    runs = [(m, L.AC_PREC_MIXED_BF16K) for m in modes]
    if fp64_plain:
        runs = [("plain_fp64", L.AC_PREC_FP64)] + runs
    inner_of = {"plain": L.AC_INNER_CHEB, "plain_fp64": L.AC_INNER_CHEB, "cnn": L.AC_INNER_CHEB_CNN,
                "cnn_cycle": L.AC_INNER_CHEB_CNN_CYCLE, "cnn_mr": L.AC_INNER_CHEB_CNN_MR}
    xref = None
    xs = {}
    for name, prec in runs:
        opts = api.Opts(precision=prec, inner=inner_of[name], p=p_inner, tol=tol, restart_m=restart, max_outer=3000)
        ws = bufs.get("solve" + name, api.ac_solve_workspace_size(prob, opts))
        x = torch.zeros(ell * nx * ny, dtype=torch.float64, device="cuda:0")
        api.ac_solve(prob, opts, bd, x, ws)  # warm-up
        best = None
        for _ in range(max(reps, 1)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = api.ac_solve(prob, opts, bd, x, ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        info["wall_s"] = best
        xs[name] = x.clone()
        if name == "plain_fp64":
            xref = xs[name]
        elif xref is not None:
            info["rel_diff_vs_fp64_plain"] = float(torch.linalg.vector_norm(x - xref) / torch.linalg.vector_norm(xref))
        out[name] = info
    # inner residuals on preconditioner inputs of the plain method (every 5th of 30)
    gains = [inner_gain(prob, cnn, v.contiguous(), p_inner, bufs)
             for v in preconditioner_inputs(prob, bd, p_inner, 30, bufs, restart=restart)[::5]]
    out["inner"] = {k: np.mean([g[k] for g in gains], axis=0).tolist() for k in ("guess", "cold", "warm")}
    out["x"] = xs
    return out


def save(path, cnn, record):
    params, c0, c1 = api.ac_cnn_get_params(cnn)
    json.dump({"params": params.tolist(), "c0": c0, "c1": c1, "record": record}, open(path, "w"))


def load(ctx, path):
    d = json.load(open(path))
    cnn = api.ac_cnn_create(ctx)
    api.ac_cnn_set_params(cnn, np.asarray(d["params"], dtype=np.float32), d["c0"], d["c1"])
    return cnn, d
