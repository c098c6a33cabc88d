// Geometric multigrid V-cycle for the shifted operators A - c I of the saddle-point
// preconditioner P_SP (Section 4): the paper applies P_D (eq. (minresprecond)) and the
// preconditioner of its real-shift CG solves with one V-cycle of a black-box algebraic
// multigrid; on these structured grids a geometric V-cycle does the same job.
//
// Vertex-centred reading of A = I + kappa (-Delta_h) (unknowns at (i + 1) h, Dirichlet
// values one spacing beyond the ends).  A dimension of n > 1 points coarsens to
// floor(n/2) points, coarse J = fine 2J + 1.  Coarse faces: the two fine faces between
// coarse neighbours in series over twice the spacing (harmonic mean / 4), the Dirichlet
// faces likewise (at the high end of an even n the last coarse point is the last fine
// point: w_b / 2), averaged along a coarsened tangential dimension over fine lines
// 2J, 2J+1, 2J+2 with weights 1/4, 1/2, 1/4.  Linear interpolation P, full weighting
// R = P^T / 2^d.  Cycle: two damped-Jacobi sweeps (omega = 0.8) from zero, coarse
// correction, two sweeps; the last level (at most 4 points) is solved exactly.  The
// cycle is a symmetric positive definite operator, as MINRES and CG need.
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr double kOmega = 0.8;

struct MgVecs {
    const double* in[kMgMaxVec];  // iterate
    const double* b[kMgMaxVec];   // right-hand side
    double* out[kMgMaxVec];
    double c[kMgMaxVec];
};

__device__ __forceinline__ double harm4(double a, double b) { return a * b / (2.0 * (a + b)); }

int grid_of(long long n) { return static_cast<int>((n + 255) / 256); }

// ---- set-up -------------------------------------------------------------------------

__global__ void fine_faces_kernel(const MgLevel L, const double* __restrict__ k) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int x = static_cast<int>(i % L.nx), y = static_cast<int>(i / L.nx);
    L.wx[i] = x < L.nx - 1 ? 0.5 * (k[i] + k[i + 1]) : 0.0;
    L.wy[i] = (L.dim == 2 && y < L.ny - 1) ? 0.5 * (k[i] + k[i + L.nx]) : 0.0;
    if (x == 0) L.bx0[y] = k[i];
    if (x == L.nx - 1) L.bx1[y] = k[i];
    if (L.dim == 2) {
        if (y == 0) L.by0[x] = k[i];
        if (y == L.ny - 1) L.by1[x] = k[i];
    } else {
        L.by0[x] = 0.0;
        L.by1[x] = 0.0;
    }
}

// Tangential average: fine lines 2J+1+d, d = -1, 0, 1, weights 1/4, 1/2, 1/4 renormalised
// to the lines inside [0, n); a dimension that was not coarsened keeps line J.
struct Tang {
    int line[3];
    double w[3];
    int cnt;
};
__device__ Tang tangential(int n, int coarsened, int J) {
    Tang t;
    t.cnt = 0;
    if (!coarsened) {
        t.line[0] = J;
        t.w[0] = 1.0;
        t.cnt = 1;
        return t;
    }
    const double wd[3] = {0.25, 0.5, 0.25};
    double tot = 0.0;
    for (int d = -1; d <= 1; ++d) {
        const int l = 2 * J + 1 + d;
        if (l >= 0 && l < n) {
            t.line[t.cnt] = l;
            t.w[t.cnt] = wd[d + 1];
            tot += wd[d + 1];
            ++t.cnt;
        }
    }
    for (int q = 0; q < t.cnt; ++q) t.w[q] /= tot;
    return t;
}

// Coarse faces of point (X, Y) of level C from level F.
__global__ void coarsen_faces_kernel(const MgLevel F, const MgLevel C) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= C.n) return;
    const int X = static_cast<int>(i % C.nx), Y = static_cast<int>(i / C.nx);
    const long long fnx = F.nx;
    // x faces, accumulated over the tangential (y) lines
    {
        const Tang t = tangential(F.ny, C.cy, Y);
        double w = 0.0, b0 = 0.0, b1 = 0.0;
        for (int q = 0; q < t.cnt; ++q) {
            const long long row = t.line[q] * fnx;
            double inner = 0.0, lo, hi;
            if (C.cx) {
                if (X < C.nx - 1) inner = harm4(F.wx[row + 2 * X + 1], F.wx[row + 2 * X + 2]);
                lo = harm4(F.bx0[t.line[q]], F.wx[row]);
                hi = (F.nx % 2 == 1) ? harm4(F.wx[row + F.nx - 2], F.bx1[t.line[q]]) : 0.5 * F.bx1[t.line[q]];
            } else {
                if (X < C.nx - 1) inner = F.wx[row + X];
                lo = F.bx0[t.line[q]];
                hi = F.bx1[t.line[q]];
            }
            w += t.w[q] * inner;
            b0 += t.w[q] * lo;
            b1 += t.w[q] * hi;
        }
        C.wx[i] = w;
        if (X == 0) C.bx0[Y] = b0;
        if (X == C.nx - 1) C.bx1[Y] = b1;
    }
    if (C.dim == 2) {
        const Tang t = tangential(F.nx, C.cx, X);
        double w = 0.0, b0 = 0.0, b1 = 0.0;
        for (int q = 0; q < t.cnt; ++q) {
            const long long col = t.line[q];
            double inner = 0.0, lo, hi;
            if (C.cy) {
                if (Y < C.ny - 1)
                    inner = harm4(F.wy[(2LL * Y + 1) * fnx + col], F.wy[(2LL * Y + 2) * fnx + col]);
                lo = harm4(F.by0[col], F.wy[col]);
                hi = (F.ny % 2 == 1) ? harm4(F.wy[(F.ny - 2LL) * fnx + col], F.by1[col]) : 0.5 * F.by1[col];
            } else {
                if (Y < C.ny - 1) inner = F.wy[static_cast<long long>(Y) * fnx + col];
                lo = F.by0[col];
                hi = F.by1[col];
            }
            w += t.w[q] * inner;
            b0 += t.w[q] * lo;
            b1 += t.w[q] * hi;
        }
        C.wy[i] = w;
        if (Y == 0) C.by0[X] = b0;
        if (Y == C.ny - 1) C.by1[X] = b1;
    } else {
        C.wy[i] = 0.0;
        C.by0[X] = 0.0;
        C.by1[X] = 0.0;
    }
}

__global__ void diag_kernel(const MgLevel L) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int x = static_cast<int>(i % L.nx), y = static_cast<int>(i / L.nx);
    double d = 1.0;
    d += x < L.nx - 1 ? L.wx[i] : 0.0;
    d += x > 0 ? L.wx[i - 1] : 0.0;
    d += x == 0 ? L.bx0[y] : 0.0;
    d += x == L.nx - 1 ? L.bx1[y] : 0.0;
    if (L.dim == 2) {
        d += y < L.ny - 1 ? L.wy[i] : 0.0;
        d += y > 0 ? L.wy[i - L.nx] : 0.0;
        d += y == 0 ? L.by0[x] : 0.0;
        d += y == L.ny - 1 ? L.by1[x] : 0.0;
    }
    L.diag[i] = d;
}

// ---- cycle kernels (grid: points x vectors) --------------------------------------------

// (A - c I) u at point i
__device__ __forceinline__ double apply_at(const MgLevel& L, const double* __restrict__ u, long long i, int x, int y,
                                           double c) {
    double a = (L.diag[i] - c) * u[i];
    if (x < L.nx - 1) a -= L.wx[i] * u[i + 1];
    if (x > 0) a -= L.wx[i - 1] * u[i - 1];
    if (L.dim == 2) {
        if (y < L.ny - 1) a -= L.wy[i] * u[i + L.nx];
        if (y > 0) a -= L.wy[i - L.nx] * u[i - L.nx];
    }
    return a;
}

// FIRST: out = omega b / d (the sweep from zero); else out = in + omega (b - (A - cI) in) / d
template <bool FIRST>
__global__ void jacobi_kernel(const MgLevel L, const MgVecs v) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int q = blockIdx.y;
    const double c = v.c[q];
    const double d = L.diag[i] - c;
    if (FIRST) {
        v.out[q][i] = kOmega * v.b[q][i] / d;
        return;
    }
    const int x = static_cast<int>(i % L.nx), y = static_cast<int>(i / L.nx);
    v.out[q][i] = v.in[q][i] + kOmega * (v.b[q][i] - apply_at(L, v.in[q], i, x, y, c)) / d;
}

__global__ void residual_kernel(const MgLevel L, const MgVecs v) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int q = blockIdx.y;
    const int x = static_cast<int>(i % L.nx), y = static_cast<int>(i / L.nx);
    v.out[q][i] = v.b[q][i] - apply_at(L, v.in[q], i, x, y, v.c[q]);
}

// coarse out = R fine in: per coarsened dimension fine 2J (1/2), 2J+1 (1), 2J+2 (1/2),
// divided by 2 per coarsened dimension
__global__ void restrict_kernel(const MgLevel F, const MgLevel C, const MgVecs v) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= C.n) return;
    const int q = blockIdx.y;
    const int X = static_cast<int>(i % C.nx), Y = static_cast<int>(i / C.nx);
    const double* __restrict__ in = v.in[q];
    const double wd[3] = {0.5, 1.0, 0.5};
    double acc = 0.0;
    for (int dy = 0; dy < (C.cy ? 3 : 1); ++dy) {
        const int y = C.cy ? 2 * Y + dy : Y;
        if (y >= F.ny) continue;
        const double wy = C.cy ? wd[dy] : 1.0;
        for (int dx = 0; dx < (C.cx ? 3 : 1); ++dx) {
            const int x = C.cx ? 2 * X + dx : X;
            if (x >= F.nx) continue;
            const double wx = C.cx ? wd[dx] : 1.0;
            acc += wy * wx * in[static_cast<long long>(y) * F.nx + x];
        }
    }
    v.out[q][i] = acc / static_cast<double>(1 << (C.cx + C.cy));
}

// fine out += P coarse in
__global__ void prolong_add_kernel(const MgLevel F, const MgLevel C, const MgVecs v) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= F.n) return;
    const int q = blockIdx.y;
    const int x = static_cast<int>(i % F.nx), y = static_cast<int>(i / F.nx);
    int jx[2], jy[2];
    double wx[2], wy[2];
    int nx = 0, ny = 0;
    if (!C.cx) {
        jx[0] = x;
        wx[0] = 1.0;
        nx = 1;
    } else if (x % 2 == 1) {
        jx[0] = (x - 1) / 2;
        wx[0] = 1.0;
        nx = 1;
    } else {
        if (x / 2 - 1 >= 0) {
            jx[nx] = x / 2 - 1;
            wx[nx++] = 0.5;
        }
        if (x / 2 < C.nx) {
            jx[nx] = x / 2;
            wx[nx++] = 0.5;
        }
    }
    if (!C.cy) {
        jy[0] = y;
        wy[0] = 1.0;
        ny = 1;
    } else if (y % 2 == 1) {
        jy[0] = (y - 1) / 2;
        wy[0] = 1.0;
        ny = 1;
    } else {
        if (y / 2 - 1 >= 0) {
            jy[ny] = y / 2 - 1;
            wy[ny++] = 0.5;
        }
        if (y / 2 < C.ny) {
            jy[ny] = y / 2;
            wy[ny++] = 0.5;
        }
    }
    const double* __restrict__ e = v.in[q];
    double acc = 0.0;
    for (int b = 0; b < ny; ++b)
        for (int a = 0; a < nx; ++a) acc += wy[b] * wx[a] * e[static_cast<long long>(jy[b]) * C.nx + jx[a]];
    v.out[q][i] += acc;
}

// Exact solve on a level of at most 4 points: one thread per vector, Gaussian
// elimination (A - c I is symmetric positive definite).
__global__ void coarsest_kernel(const MgLevel L, const MgVecs v, int nv) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nv) return;
    const int n = static_cast<int>(L.n);
    double M[4][4], r[4];
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) M[a][b] = 0.0;
        r[a] = v.b[q][a];
    }
    for (int a = 0; a < n; ++a) {
        const int x = a % L.nx, y = a / L.nx;
        M[a][a] = L.diag[a] - v.c[q];
        if (x < L.nx - 1) {
            M[a][a + 1] = -L.wx[a];
            M[a + 1][a] = -L.wx[a];
        }
        if (L.dim == 2 && y < L.ny - 1) {
            M[a][a + L.nx] = -L.wy[a];
            M[a + L.nx][a] = -L.wy[a];
        }
    }
    for (int k = 0; k < n; ++k)
        for (int a = k + 1; a < n; ++a) {
            const double f = M[a][k] / M[k][k];
            for (int b = k; b < n; ++b) M[a][b] -= f * M[k][b];
            r[a] -= f * r[k];
        }
    for (int a = n - 1; a >= 0; --a) {
        double t = r[a];
        for (int b = a + 1; b < n; ++b) t -= M[a][b] * r[b];
        r[a] = t / M[a][a];
    }
    for (int a = 0; a < n; ++a) v.out[q][a] = r[a];
}

}  // namespace

int mg_plan(int dim, int nx, int ny, MgLevel* out) {
    if (dim == 1) ny = 1;
    int nl = 0;
    int cx = 0, cy = 0;
    while (true) {
        MgLevel L{};
        L.nx = nx;
        L.ny = ny;
        L.dim = dim;
        L.cx = cx;
        L.cy = cy;
        L.n = static_cast<long long>(nx) * ny;
        if (nl >= kMgMaxLevels) return -1;
        out[nl++] = L;
        if (L.n <= 4) break;
        cx = nx > 1;
        cy = dim == 2 && ny > 1;
        if (cx) nx /= 2;
        if (cy) ny /= 2;
    }
    return nl;
}

size_t mg_level_doubles(const MgLevel& L) {
    return 3 * static_cast<size_t>(L.n) + 2 * static_cast<size_t>(L.nx) + 2 * static_cast<size_t>(L.ny);
}

hipError_t mg_build(const MgHierarchy& h, const double* kappa, hipStream_t s) {
    hipLaunchKernelGGL(fine_faces_kernel, dim3(grid_of(h.lev[0].n)), dim3(256), 0, s, h.lev[0], kappa);
    hipLaunchKernelGGL(diag_kernel, dim3(grid_of(h.lev[0].n)), dim3(256), 0, s, h.lev[0]);
    for (int l = 1; l < h.nlev; ++l) {
        hipLaunchKernelGGL(coarsen_faces_kernel, dim3(grid_of(h.lev[l].n)), dim3(256), 0, s, h.lev[l - 1], h.lev[l]);
        hipLaunchKernelGGL(diag_kernel, dim3(grid_of(h.lev[l].n)), dim3(256), 0, s, h.lev[l]);
    }
    return hipGetLastError();
}

size_t mg_scratch_doubles(const MgHierarchy& h, int nv) {
    // level 0: one work vector per right-hand side; coarser levels: b, u, t
    size_t d = static_cast<size_t>(nv) * h.lev[0].n;
    for (int l = 1; l < h.nlev; ++l) d += 3 * static_cast<size_t>(nv) * h.lev[l].n;
    return d;
}

hipError_t mg_vcycle(const MgHierarchy& h, int nv, const double* const* b, double* const* u, const double* c,
                     double* scratch, hipStream_t s) {
    if (nv < 1 || nv > kMgMaxVec || h.nlev < 1) return hipErrorInvalidValue;
    // per level: B (right-hand sides), U (work), T (result)
    const double* B[kMgMaxLevels][kMgMaxVec];
    double* U[kMgMaxLevels][kMgMaxVec];
    double* T[kMgMaxLevels][kMgMaxVec];
    double* p = scratch;
    for (int q = 0; q < nv; ++q) {
        B[0][q] = b[q];
        T[0][q] = u[q];
        U[0][q] = p + static_cast<size_t>(q) * h.lev[0].n;
    }
    p += static_cast<size_t>(nv) * h.lev[0].n;
    for (int l = 1; l < h.nlev; ++l) {
        const size_t n = h.lev[l].n;
        for (int q = 0; q < nv; ++q) {
            B[l][q] = p + q * n;
            U[l][q] = p + (nv + q) * n;
            T[l][q] = p + (2 * nv + q) * n;
        }
        p += 3 * nv * n;
    }
    auto vecs = [&](int l, double* const* in, const double* const* rhs, double* const* out) {
        MgVecs v{};
        for (int q = 0; q < nv; ++q) {
            v.in[q] = in ? in[q] : nullptr;
            v.b[q] = rhs ? rhs[q] : nullptr;
            v.out[q] = out[q];
            v.c[q] = c[q];
        }
        (void)l;
        return v;
    };
    // down the hierarchy
    for (int l = 0; l < h.nlev - 1; ++l) {
        const MgLevel& L = h.lev[l];
        const dim3 g(grid_of(L.n), nv);
        hipLaunchKernelGGL(jacobi_kernel<true>, g, dim3(256), 0, s, L, vecs(l, nullptr, B[l], U[l]));
        hipLaunchKernelGGL(jacobi_kernel<false>, g, dim3(256), 0, s, L, vecs(l, U[l], B[l], T[l]));
        hipLaunchKernelGGL(residual_kernel, g, dim3(256), 0, s, L, vecs(l, T[l], B[l], U[l]));
        double* const* Bn = const_cast<double* const*>(B[l + 1]);
        hipLaunchKernelGGL(restrict_kernel, dim3(grid_of(h.lev[l + 1].n), nv), dim3(256), 0, s, L, h.lev[l + 1],
                           vecs(l, U[l], nullptr, Bn));
    }
    const int last = h.nlev - 1;
    hipLaunchKernelGGL(coarsest_kernel, dim3(1), dim3(64), 0, s, h.lev[last], vecs(last, nullptr, B[last], T[last]), nv);
    // and back up
    for (int l = h.nlev - 2; l >= 0; --l) {
        const MgLevel& L = h.lev[l];
        const dim3 g(grid_of(L.n), nv);
        hipLaunchKernelGGL(prolong_add_kernel, g, dim3(256), 0, s, L, h.lev[l + 1], vecs(l, T[l + 1], nullptr, T[l]));
        hipLaunchKernelGGL(jacobi_kernel<false>, g, dim3(256), 0, s, L, vecs(l, T[l], B[l], U[l]));
        hipLaunchKernelGGL(jacobi_kernel<false>, g, dim3(256), 0, s, L, vecs(l, U[l], B[l], T[l]));
    }
    return hipGetLastError();
}

}  // namespace ac
