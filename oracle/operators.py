"""Spatial operator A, all-at-once operator, sequential solve, spectral intervals.

Readings of the paper used here:
* The paper's operator is A = I - (nu/h^2) L with L the five-point Dirichlet
  Laplacian (Section 5, eq. (IminusLap)).  With a cell-centred coefficient
  kappa this generalises to (A u)_i = u_i + sum_faces kappa_f (u_i - u_nb),
  with face value kappa_f = (kappa_i + kappa_nb)/2; a Dirichlet boundary face
  uses the cell's own kappa and a zero ghost value.  A constant kappa gives
  exactly I + kappa (-Delta_h), i.e. the paper's operator with
  kappa = nu / h^2.
* 1D grids have faces in x only; 2D grids in x and y.  Periodic wrap-around is
  provided for the closed-form DFT check only.

Pins (tests/test_oracle_operators.py): the constant-coefficient spectrum and
sine eigenvectors of Appendix A, the periodic DFT eigenvalues, the all-at-once
solve against the sequential chain A x_{k+1} = x_k (Section 1), the closed-form
(sine-transform) chain against the sparse direct chain and against the assembled
all-at-once matrix, Gershgorin / Rayleigh bounds against eigsh.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _neighbours(nx: int, ny: int, dim: int, periodic: bool):
    """Yield (cell index, neighbour index or -1) for every face direction."""
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    dirs = [(1, 0), (-1, 0)]
    if dim == 2:
        dirs += [(0, 1), (0, -1)]
    for dx, dy in dirs:
        jx = ix + dx
        jy = iy + dy
        if periodic:
            jx %= nx
            jy %= ny
            nb = jy * nx + jx
        else:
            inside = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny)
            nb = np.where(inside, jy * nx + jx, -1)
        yield np.arange(nx * ny), nb


def build_A(dim: int, nx: int, ny: int, kappa, bc: str = "dirichlet") -> sp.csr_matrix:
    """Sparse FP64 A = I + sum_f kappa_f (e_i - e_nb)(...)  (see module docstring).

    ``kappa`` is a scalar or an array of length N = nx*ny (ny = 1 when dim = 1).
    """
    if dim == 1:
        ny = 1
    n = nx * ny
    kap = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (n,))
    periodic = bc == "periodic"
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.ones(n)]
    for i, nb in _neighbours(nx, ny, dim, periodic):
        interior = nb >= 0
        kf = np.where(interior, 0.5 * (kap + kap[np.where(interior, nb, 0)]), kap)
        # diagonal contribution kappa_f
        rows.append(i)
        cols.append(i)
        vals.append(kf)
        # off-diagonal -kappa_f towards the neighbour (absent at a Dirichlet face)
        rows.append(i[interior])
        cols.append(nb[interior])
        vals.append(-kf[interior])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A.tocsr()


def shift_matrix(ell: int) -> sp.csr_matrix:
    """S: ones on the first sub-diagonal (ell x ell)."""
    return sp.diags([np.ones(ell - 1)], [-1], shape=(ell, ell), format="csr")


def build_calA(A: sp.spmatrix, ell: int) -> sp.csr_matrix:
    """All-at-once matrix of eq. (1): A on the block diagonal, -I below it."""
    n = A.shape[0]
    return (sp.kron(sp.identity(ell), A) - sp.kron(shift_matrix(ell), sp.identity(n))).tocsr()


def apply_calA(A: sp.spmatrix, x: np.ndarray, ell: int) -> np.ndarray:
    """y_k = A x_k - x_{k-1} (x_0 := 0), block by block (eq. (1))."""
    n = A.shape[0]
    X = x.reshape(ell, n)
    Y = np.empty_like(X, dtype=np.result_type(x, np.float64))
    for k in range(ell):
        Y[k] = A @ X[k]
        if k > 0:
            Y[k] -= X[k - 1]
    return Y.reshape(-1)


def sequential_solve(A: sp.spmatrix, b: np.ndarray, ell: int) -> np.ndarray:
    """Solve the all-at-once system as the chain A x_1 = b_1, A x_k = b_k + x_{k-1}
    (Section 1: the implicit diffusion operator as a sequence of ell solves)."""
    n = A.shape[0]
    lu = spla.splu(A.tocsc())
    B = b.reshape(ell, n)
    X = np.empty((ell, n))
    prev = np.zeros(n)
    for k in range(ell):
        X[k] = lu.solve(B[k] + prev)
        prev = X[k]
    return X.reshape(-1)


def sequential_solve_closed_form(dim: int, nx: int, ny: int, kappa: float, b: np.ndarray, ell: int) -> np.ndarray:
    """The chain of sequential_solve for a constant coefficient on a Dirichlet grid, at
    any size in O(l N log N): the orthonormal DST-I per axis diagonalises A (Appendix A:
    sine eigenvectors, eigenvalues mu = 1 + 4 kappa sum_d sin^2(.)), so in mode space
    every link of the chain A x_1 = b_1, A x_k = b_k + x_{k-1} (Section 1) is a division
    by mu."""
    if dim == 1:
        ny = 1
    n = nx * ny
    shape = (nx,) if dim == 1 else (ny, nx)
    axes = (0,) if dim == 1 else (0, 1)
    mu = dirichlet_eigs(dim, nx, ny, float(kappa))
    B = np.asarray(b, dtype=np.float64).reshape(ell, n)
    X = np.empty((ell, n))
    prev_hat = np.zeros(shape)
    for k in range(ell):
        rhs_hat = sfft.dstn(B[k].reshape(shape), type=1, axes=axes, norm="ortho") + prev_hat
        prev_hat = rhs_hat / mu
        X[k] = sfft.idstn(prev_hat, type=1, axes=axes, norm="ortho").reshape(-1)
    return X.reshape(-1)


# ---------------------------------------------------------------------------
# Varying diagonal blocks (Conclusions): calA = blockdiag(A_1, ..., A_l) - S (x) I,
# preconditioned through a representative block A_hat.

def build_calA_blocks(As) -> sp.csr_matrix:
    """All-at-once matrix with block k on the diagonal and -I below it."""
    ell, n = len(As), As[0].shape[0]
    return (sp.block_diag(As) - sp.kron(shift_matrix(ell), sp.identity(n))).tocsr()


def apply_calA_blocks(As, x: np.ndarray) -> np.ndarray:
    """y_k = A_k x_k - x_{k-1} (x_0 := 0)."""
    ell, n = len(As), As[0].shape[0]
    X = x.reshape(ell, n)
    Y = np.empty_like(X, dtype=np.float64)
    for k in range(ell):
        Y[k] = As[k] @ X[k]
        if k > 0:
            Y[k] -= X[k - 1]
    return Y.reshape(-1)


def sequential_solve_blocks(As, b: np.ndarray) -> np.ndarray:
    """The chain A_1 x_1 = b_1, A_k x_k = b_k + x_{k-1}."""
    ell, n = len(As), As[0].shape[0]
    B = b.reshape(ell, n)
    X = np.empty((ell, n))
    prev = np.zeros(n)
    for k in range(ell):
        X[k] = spla.spsolve(As[k].tocsc(), B[k] + prev)
        prev = X[k]
    return X.reshape(-1)


def mean_block_kappa(kappas: np.ndarray) -> np.ndarray:
    """Cell coefficients of the representative block: the pointwise mean of the
    blocks' coefficients.  A is affine in kappa (face values are means of cell
    values), so A(mean kappa) is the mean of the blocks A_k."""
    return np.asarray(kappas, dtype=np.float64).reshape(len(kappas), -1).mean(axis=0)


def dirichlet_eigs_1d(n: int, kappa: float) -> np.ndarray:
    """Eigenvalues 1 + 4 kappa sin^2(k pi / (2(n+1))), k = 1..n (Appendix A, 1D factor)."""
    k = np.arange(1, n + 1)
    return 1.0 + 4.0 * kappa * np.sin(k * np.pi / (2 * (n + 1))) ** 2


def dirichlet_eigs(dim: int, nx: int, ny: int, kappa: float) -> np.ndarray:
    """Appendix A: mu_{i,j} = 1 + 4 kappa (sin^2(i pi/(2(nx+1))) + sin^2(j pi/(2(ny+1))))
    with kappa = nu/h^2; returned as an (ny, nx) array (1D: length nx)."""
    sx = np.sin(np.arange(1, nx + 1) * np.pi / (2 * (nx + 1))) ** 2
    if dim == 1:
        return 1.0 + 4.0 * kappa * sx
    sy = np.sin(np.arange(1, ny + 1) * np.pi / (2 * (ny + 1))) ** 2
    return 1.0 + 4.0 * kappa * (sy[:, None] + sx[None, :])


def periodic_eigs(dim: int, nx: int, ny: int, kappa: float) -> np.ndarray:
    """Eigenvalues 1 + 4 kappa sum_d sin^2(pi k_d / n_d) of the periodic operator, laid
    out like numpy's fft2 output ((ny, nx), or (nx,) in 1D)."""
    sx = np.sin(np.pi * np.arange(nx) / nx) ** 2
    if dim == 1:
        return 1.0 + 4.0 * kappa * sx
    sy = np.sin(np.pi * np.arange(ny) / ny) ** 2
    return 1.0 + 4.0 * kappa * (sy[:, None] + sx[None, :])


def sine_vector(n: int, j: int) -> np.ndarray:
    """Normalised eigenvector V_j = sqrt(2/(n+1)) (sin(i j pi/(n+1)))_{i=1..n} (Appendix A)."""
    i = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(i * j * np.pi / (n + 1))


def min_laplacian_eig(dim: int, nx: int, ny: int, bc: str = "dirichlet") -> float:
    """Smallest eigenvalue of -Delta_h (integer stencil): 4 sin^2(pi/(2(n+1))) per axis
    for Dirichlet, 0 for periodic."""
    if bc == "periodic":
        return 0.0
    v = 4.0 * np.sin(np.pi / (2 * (nx + 1))) ** 2
    if dim == 2:
        v += 4.0 * np.sin(np.pi / (2 * (ny + 1))) ** 2
    return float(v)


def spectral_interval(dim: int, nx: int, ny: int, kappa, bc: str = "dirichlet"):
    """Rigorous enclosing interval [mu_lo, mu_hi] of the spectrum of A.

    mu_hi: Gershgorin, max over rows of (diagonal + sum |off-diagonal|).
    mu_lo: 1 + min(kappa) * lambda_min(-Delta_h), valid because every face
    coefficient is at least min(kappa), so u^T (A - I) u >= min(kappa) u^T (-Delta_h) u.
    For a constant kappa both reduce to the closed forms of Appendix A except that
    the Gershgorin value 1 + 2 * (2 dim) kappa is replaced by the exact maximum.
    """
    A = build_A(dim, nx, ny, kappa, bc)
    centre = A.diagonal()
    radius = abs(A).sum(axis=1).A1 - np.abs(centre)
    gersh = float(np.max(centre + radius))
    kap = np.asarray(kappa, dtype=np.float64)
    mu_lo = 1.0 + float(np.min(kap)) * min_laplacian_eig(dim, nx, ny if dim == 2 else 1, bc)
    return mu_lo, gersh


def constant_interval(dim: int, nx: int, ny: int, kappa: float, bc: str = "dirichlet"):
    """Exact [mu_min, mu_max] for a constant coefficient (Appendix A / periodic DFT)."""
    ev = dirichlet_eigs(dim, nx, ny, kappa) if bc == "dirichlet" else periodic_eigs(dim, nx, ny, kappa)
    return float(ev.min()), float(ev.max())
