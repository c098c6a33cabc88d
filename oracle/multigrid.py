"""Geometric multigrid V-cycle for the shifted operator A - c I (oracle, test infrastructure).

The paper applies the block preconditioner P_D of Section 4 (eq. (minresprecond)) and the
preconditioner of its real-shift CG solves with one V-cycle of an algebraic multigrid
code used as a black box (Section 5).  No multigrid is specified there, so this module
defines the one the library implements for its structured grids: a geometric V-cycle on
the vertex-centred reading of the operator (unknowns at the points (i + 1) h, Dirichlet
values one spacing beyond the first and last points, as for I + kappa (-Delta_h)).
Nothing here is a paper pin; the tests pin it to properties that fix it (symmetry and
positivity of the V-cycle, the fine level equal to the operators module's A, an exact
solve on the coarsest level, prolongation reproducing linear functions, a contraction
bound).

Definition (every level stores face coefficients; the diagonal is 1 + the sum of a
point's face coefficients, so A_l u = u + sum_f w_f (u_i - u_nb) with zero outside):
* Level 0 is A: interior face (kappa_i + kappa_j)/2, Dirichlet face kappa_i.
* A dimension with n > 1 points is coarsened to n_c = floor(n/2) points: coarse point J
  is fine point 2J + 1.  Along the normal of a face, the two fine faces between coarse
  neighbours act in series over twice the spacing: w = harmonic mean / 4 = ab/(2(a+b)).
  At a boundary the fine Dirichlet face and the first interior face combine the same
  way, except at the high end of an even n, where the last coarse point is the last fine
  point and its Dirichlet face is w_b/2 (spacing 2h on one side, h on the other).
  Along the tangential direction of a coarsened dimension the result is averaged over
  the fine lines 2J, 2J+1, 2J+2 with weights 1/4, 1/2, 1/4 (renormalised at the ends).
  Coarsening stops at a level of at most 4 points.
* Prolongation P is linear interpolation per coarsened dimension (fine point 2J + 1
  takes coarse J; fine 2J takes half of coarse J - 1 and half of coarse J, zero outside),
  the tensor product across dimensions; restriction R = P^T / 2^d, d = the number of
  coarsened dimensions (full weighting).
* V-cycle for b: on the coarsest level the exact solution of (A_l - c I) u = b;
  otherwise NU damped-Jacobi sweeps u <- u + OMEGA D^{-1} (b - (A_l - c I) u) from u = 0
  (D the diagonal of A_l - c I), the coarse correction u <- u + P V(R (b - (A_l - c I) u)),
  and NU more sweeps.  The same sweeps before and after and R proportional to P^T make
  the cycle a symmetric operator.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

OMEGA = 0.8
NU = 2


@dataclass
class Level:
    nx: int
    ny: int
    dim: int
    wx: np.ndarray   # (ny, nx-1) interior x faces: (y, x) -- (y, x+1)
    wy: np.ndarray   # (ny-1, nx) interior y faces: (y, x) -- (y+1, x); empty for dim 1
    bx0: np.ndarray  # (ny,) Dirichlet face left of column 0
    bx1: np.ndarray  # (ny,) right of column nx-1
    by0: np.ndarray  # (nx,) below row 0 (dim 2)
    by1: np.ndarray  # (nx,) above row ny-1 (dim 2)
    cx: bool = False  # this level was made by coarsening x (resp. y) of the previous one
    cy: bool = False

    def diag(self) -> np.ndarray:
        d = np.ones((self.ny, self.nx))
        d[:, :-1] += self.wx
        d[:, 1:] += self.wx
        d[:, 0] += self.bx0
        d[:, -1] += self.bx1
        if self.dim == 2:
            d[:-1, :] += self.wy
            d[1:, :] += self.wy
            d[0, :] += self.by0
            d[-1, :] += self.by1
        return d.reshape(-1)


def fine_level(dim: int, nx: int, ny: int, kappa) -> Level:
    if dim == 1:
        ny = 1
    k = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (nx * ny,)).reshape(ny, nx)
    wx = 0.5 * (k[:, :-1] + k[:, 1:])
    if dim == 2:
        wy = 0.5 * (k[:-1, :] + k[1:, :])
        by0, by1 = k[0, :].copy(), k[-1, :].copy()
    else:
        wy = np.zeros((0, nx))
        by0 = by1 = np.zeros(nx)
    return Level(nx, ny, dim, wx, wy, k[:, 0].copy(), k[:, -1].copy(), by0, by1)


def _harm4(a, b):
    """Two faces in series over twice the spacing: harmonic mean / 4."""
    return a * b / (2.0 * (a + b))


def _tangential(n: int, coarsened: bool, J: int):
    """Fine lines and weights averaged along a face's tangential direction."""
    if not coarsened:
        return [(J, 1.0)]
    pts = [(2 * J + 1 + d, w) for d, w in ((-1, 0.25), (0, 0.5), (1, 0.25)) if 0 <= 2 * J + 1 + d < n]
    tot = sum(w for _, w in pts)
    return [(i, w / tot) for i, w in pts]


def _normal_faces(w_int, b_lo, b_hi, n: int, coarsened: bool):
    """Coarse faces along one line from the fine ones: interior (n_c - 1), low and high
    Dirichlet faces.  w_int has n - 1 entries, b_lo / b_hi are scalars."""
    if not coarsened:
        return np.asarray(w_int, dtype=np.float64).copy(), b_lo, b_hi
    nc = n // 2
    inner = np.array([_harm4(w_int[2 * J + 1], w_int[2 * J + 2]) for J in range(nc - 1)])
    lo = _harm4(b_lo, w_int[0])
    hi = _harm4(w_int[n - 2], b_hi) if n % 2 == 1 else 0.5 * b_hi
    return inner, lo, hi


def coarsen(f: Level) -> Level:
    cx = f.nx > 1
    cy = f.dim == 2 and f.ny > 1
    nxc = f.nx // 2 if cx else f.nx
    nyc = f.ny // 2 if cy else f.ny
    wx = np.zeros((nyc, max(nxc - 1, 0)))
    bx0, bx1 = np.zeros(nyc), np.zeros(nyc)
    for Y in range(nyc):
        for y, wt in _tangential(f.ny, cy, Y):
            inner, lo, hi = _normal_faces(f.wx[y], f.bx0[y], f.bx1[y], f.nx, cx)
            wx[Y] += wt * inner
            bx0[Y] += wt * lo
            bx1[Y] += wt * hi
    if f.dim == 2:
        wy = np.zeros((max(nyc - 1, 0), nxc))
        by0, by1 = np.zeros(nxc), np.zeros(nxc)
        for X in range(nxc):
            for x, wt in _tangential(f.nx, cx, X):
                inner, lo, hi = _normal_faces(f.wy[:, x], f.by0[x], f.by1[x], f.ny, cy)
                wy[:, X] += wt * inner
                by0[X] += wt * lo
                by1[X] += wt * hi
    else:
        wy = np.zeros((0, nxc))
        by0 = by1 = np.zeros(nxc)
    return Level(nxc, nyc, f.dim, wx, wy, bx0, bx1, by0, by1, cx, cy)


def hierarchy(dim: int, nx: int, ny: int, kappa) -> list[Level]:
    levels = [fine_level(dim, nx, ny, kappa)]
    while levels[-1].nx * levels[-1].ny > 4:
        levels.append(coarsen(levels[-1]))
    return levels


def level_matrix(L: Level, c: float = 0.0) -> sp.csr_matrix:
    """Sparse A_l - c I assembled from the face coefficients."""
    n = L.nx * L.ny
    idx = np.arange(n).reshape(L.ny, L.nx)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [L.diag() - c]
    if L.nx > 1:
        a, b = idx[:, :-1].ravel(), idx[:, 1:].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-L.wx.ravel(), -L.wx.ravel()]
    if L.dim == 2 and L.ny > 1:
        a, b = idx[:-1, :].ravel(), idx[1:, :].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-L.wy.ravel(), -L.wy.ravel()]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def _interp_1d(n: int, nc: int, coarsened: bool) -> sp.csr_matrix:
    if not coarsened:
        return sp.identity(n, format="csr")
    rows, cols, vals = [], [], []
    for i in range(n):
        if i % 2 == 1:
            rows.append(i)
            cols.append((i - 1) // 2)
            vals.append(1.0)
        else:
            for J in (i // 2 - 1, i // 2):
                if 0 <= J < nc:
                    rows.append(i)
                    cols.append(J)
                    vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def prolongation(f: Level, c: Level) -> sp.csr_matrix:
    """P (fine x coarse); the grid index is y * nx + x, so P = P_y (x) P_x."""
    return sp.kron(_interp_1d(f.ny, c.ny, c.cy), _interp_1d(f.nx, c.nx, c.cx), format="csr")


def restriction(f: Level, c: Level) -> sp.csr_matrix:
    d = int(c.cx) + int(c.cy)
    return (prolongation(f, c).T / float(2 ** d)).tocsr()


def vcycle(levels: list[Level], b: np.ndarray, c: float, l: int = 0, nu: int = NU, omega: float = OMEGA):
    """One V-cycle for (A_l - c I) u = b from u = 0 (see the module docstring)."""
    A = level_matrix(levels[l], c)
    if l == len(levels) - 1:
        return spla.spsolve(A.tocsc(), b) if A.shape[0] > 1 else b / A.toarray()[0, 0]
    D = A.diagonal()
    u = np.zeros_like(b)
    for _ in range(nu):
        u = u + omega * (b - A @ u) / D
    P = prolongation(levels[l], levels[l + 1])
    R = restriction(levels[l], levels[l + 1])
    u = u + P @ vcycle(levels, R @ (b - A @ u), c, l + 1, nu, omega)
    for _ in range(nu):
        u = u + omega * (b - A @ u) / D
    return u
