"""Decomposition of the fused Chebyshev sweeps (blocks of two and three steps): a model of
the library's block tiling (strips of 64*vx computed columns advancing by
64*vx - 2*(depth-1), chunks of h rows, the XCD-aware block remap) and of the kernels'
ownership rule (a strip writes its inner columns [x0 + depth-1, x0 + 64*vx - depth],
the first strip from column 0).  Every grid point must be written by exactly one wave,
and every lane's vector of vx points must lie inside the grid or wholly outside it, for
ragged grids, both depths, both widths and several chunk heights and block sizes.
Host-side logic only (no GPU)."""

import numpy as np
import pytest


def _tiles(nx, ny, vx, h, wpb, depth):
    w = 64 * vx
    stride = w - 2 * (depth - 1)
    nsx = (nx - (depth - 1) + stride - 1) // stride
    h = min(h, ny)
    ncy = (ny + h - 1) // h
    tiles = nsx * ncy
    nb = (tiles + wpb - 1) // wpb
    per = nb >> 3
    full = per << 3
    for bid in range(nb):
        b2 = (bid & 7) * per + (bid >> 3) if bid < full else bid
        for wave in range(wpb):
            t = b2 * wpb + wave
            if t < tiles:
                yield t, (t % nsx) * stride, (t // nsx) * h, min((t // nsx) * h + h, ny)


def _coverage(nx, ny, vx, h, wpb, depth):
    w = 64 * vx
    seen = set()
    count = np.zeros((ny, nx), dtype=np.int64)
    for t, x0, y0, y1 in _tiles(nx, ny, vx, h, wpb, depth):
        assert t not in seen
        seen.add(t)
        lo, hi = x0 + (depth - 1), x0 + w - depth
        for lane in range(64):
            xb = x0 + lane * vx
            if xb >= nx:
                continue
            assert xb + vx - 1 < nx  # a lane's vector is wholly inside the grid
            for v in range(vx):
                c = xb + v
                if (c >= lo or x0 == 0) and c <= hi:
                    count[y0:y1, c] += 1
    return count


@pytest.mark.parametrize("depth", [2, 3])
@pytest.mark.parametrize("vx", [1, 2])
def test_every_point_written_once(depth, vx):
    for nx in [3, 4, 5, 63, 64, 65, 124, 125, 126, 127, 128, 130, 248, 250, 252, 254, 256, 372, 500]:
        if vx == 2 and (nx % 2 or nx < 128):
            continue  # two points per lane only on even grids at least 128 wide
        if nx < depth + 1:
            continue  # pairs need nx >= 3, blocks of three nx >= 4
        for ny in [1, 2, 7, 17]:
            for h in [1, 4, 9, 12]:
                for wpb in [1, 4]:
                    c = _coverage(nx, ny, vx, h, wpb, depth)
                    assert (c == 1).all(), (nx, ny, vx, h, wpb, depth, c.min(), c.max())


def test_full_size_decomposition():
    """The benchmark grid at its automatic tiling: 2048^2, 12 rows per wave, 4 waves."""
    for depth in (2, 3):
        c = _coverage(2048, 48, 2, 12, 4, depth)
        assert (c == 1).all()
