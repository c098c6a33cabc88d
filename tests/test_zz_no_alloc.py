"""ac_apply_prec_noalloc (the entry point for callers that cannot allocate): through the
C ABI against ac_apply_prec on the same inputs.  Both run the same kernels on the same
data, so the outputs must agree bit for bit; two calls in a row, the second on a smaller
problem (the fixed scratch keeps the first call's contents), in both inner precisions,
then a problem too large for the scratch (rejected on the host)."""

import numpy as np
import pytest
import torch

from paper_2506_03947_amd import api
from synth import lognormal_kappa, random_block_vector
from tests import gpu_util as G

L = api.L
pytestmark = pytest.mark.gpu


def _pair(p, opts, r):
    rd = G.dev(r)
    z_ref = torch.full_like(rd, np.nan)
    api.ac_apply_prec(p, opts, rd, z_ref, api.workspace(api.ac_prec_workspace_size(p, opts)))
    z = torch.full_like(rd, np.nan)
    api.ac_apply_prec_noalloc(p, opts, rd, z)
    return G.host(z), G.host(z_ref)


@pytest.mark.parametrize("precision", [L.AC_PREC_MIXED_BF16K, L.AC_PREC_FP64])
def test_noalloc_equals_workspace_entry_point(precision):
    cases = [(2, 300, 260, 10, 20), (2, 97, 61, 6, 9)]  # second call: smaller problem
    for dim, nx, ny, ell, pp in cases:
        kap = lognormal_kappa(nx, ny, 50.0, 10.0, 1.0, seed=nx)
        p = G.problem(dim, nx, ny, kap, ell, 1e-2)
        opts = api.Opts(precision=precision, p=pp)
        assert api.ac_prec_workspace_size(p, opts) <= L.AC_NOALLOC_SCRATCH_BYTES
        r = random_block_vector(nx * ny, ell, seed=ell)
        z, z_ref = _pair(p, opts, r)
        assert np.all(np.isfinite(z))
        assert np.array_equal(z, z_ref), (nx, ny, float(np.max(np.abs(z - z_ref))))


def test_noalloc_rejects_problems_beyond_the_scratch():
    nx = ny = 1024
    p = G.problem(2, nx, ny, 50.0, 10, 1e-2)
    opts = api.Opts(precision=L.AC_PREC_MIXED_BF16K, p=10)
    assert api.ac_prec_workspace_size(p, opts) > L.AC_NOALLOC_SCRATCH_BYTES
    r = torch.zeros(10 * nx * ny, dtype=torch.float64, device="cuda:0")
    z = torch.zeros_like(r)
    with pytest.raises(RuntimeError, match="workspace"):
        api.ac_apply_prec_noalloc(p, opts, r, z)
    with pytest.raises(RuntimeError, match="unsupported|Chebyshev"):
        api.ac_apply_prec_noalloc(p, api.Opts(precision=L.AC_PREC_FP64, inner=L.AC_INNER_EXACT), r, z)
