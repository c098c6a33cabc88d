"""Helpers for the GPU parity tests: build device problems from host inputs.

Nothing here computes any part of the method; it moves host arrays to the device
and wraps the C-ABI binding.
"""

import numpy as np
import torch

from paper_2506_03947_amd import api


_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = api.ac_ctx_create(0)
    return _CTX


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def problem(dim, nx, ny, kappa, ell, alpha, bc=api.L.AC_BC_DIRICHLET, bounds=None):
    k = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (nx * ny,)).copy()
    return api.ac_problem_create(ctx(), dim, nx, ny, dev(k), ell, alpha, bc=bc, bounds=bounds)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_rel(a, b):
    """max |a - b| / max |b| (element-wise error against the largest entry)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
