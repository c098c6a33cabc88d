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
// cycle is a symmetric positive definite operator, as MINRES and CG need.  The levels of
// at most 4096 points run as one kernel (one workgroup per vector).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr double kOmega = 0.8;

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

// ---- cycle kernels -----------------------------------------------------------------
// T = double (float64 vectors and coefficients) or float (the float32 copies of the
// level arrays).  The sweeps run one thread per point over every vector of the batch
// (the level's coefficients are read once per point), two vectors at a time so that
// both vectors' loads are issued before either store.  The transfers run one thread per
// (point, vector) with the vector in blockIdx.y.

template <typename T>
struct MgVecsT {
    const T* in[kMgMaxVec];  // iterate
    const T* b[kMgMaxVec];   // right-hand side
    T* out[kMgMaxVec];
    double c[kMgMaxVec];
};

template <typename T> __device__ __forceinline__ const T* diag_of(const MgLevel& L);
template <> __device__ __forceinline__ const double* diag_of<double>(const MgLevel& L) { return L.diag; }
template <> __device__ __forceinline__ const float* diag_of<float>(const MgLevel& L) { return L.diag_f; }
template <typename T> __device__ __forceinline__ const T* wx_of(const MgLevel& L);
template <> __device__ __forceinline__ const double* wx_of<double>(const MgLevel& L) { return L.wx; }
template <> __device__ __forceinline__ const float* wx_of<float>(const MgLevel& L) { return L.wx_f; }
template <typename T> __device__ __forceinline__ const T* wy_of(const MgLevel& L);
template <> __device__ __forceinline__ const double* wy_of<double>(const MgLevel& L) { return L.wy; }
template <> __device__ __forceinline__ const float* wy_of<float>(const MgLevel& L) { return L.wy_f; }

// Coefficients of point i: A u = d u_i - e u_{i+1} - w u_{i-1} - n u_{i+nx} - s u_{i-nx}
// (a missing neighbour has coefficient 0 and is not read).
template <typename T>
struct Co {
    T d, e, w, n, s;
    bool he, hw, hn, hs;
};
template <typename T>
__device__ __forceinline__ Co<T> coef_at(const MgLevel& L, long long i, int x, int y) {
    const T* dg = diag_of<T>(L);
    const T* wx = wx_of<T>(L);
    const T* wy = wy_of<T>(L);
    Co<T> c;
    c.d = dg[i];
    c.he = x < L.nx - 1;
    c.hw = x > 0;
    c.hn = L.dim == 2 && y < L.ny - 1;
    c.hs = L.dim == 2 && y > 0;
    c.e = c.he ? wx[i] : T(0);
    c.w = c.hw ? wx[i - 1] : T(0);
    c.n = c.hn ? wy[i] : T(0);
    c.s = c.hs ? wy[i - L.nx] : T(0);
    return c;
}
// the five stencil values of an array at point i (0 for a missing neighbour)
template <typename T>
struct St {
    T c, e, w, n, s;
};
template <typename T>
__device__ __forceinline__ St<T> stencil(const Co<T>& k, const T* __restrict__ u, long long i, long long nx) {
    St<T> t;
    t.c = u[i];
    t.e = k.he ? u[i + 1] : T(0);
    t.w = k.hw ? u[i - 1] : T(0);
    t.n = k.hn ? u[i + nx] : T(0);
    t.s = k.hs ? u[i - nx] : T(0);
    return t;
}
template <typename T>
__device__ __forceinline__ T apply_st(const Co<T>& k, const St<T>& u, T c) {
    return (k.d - c) * u.c - k.e * u.e - k.w * u.w - k.n * u.n - k.s * u.s;
}

// out = in + omega (b - (A - cI) in) / (d - c)   (SWEEP)   or   out = b - (A - cI) in
template <typename T, bool SWEEP>
__global__ void sweep_kernel(const MgLevel L, const MgVecsT<T> v, int nv) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int ii = static_cast<int>(i), x = ii % L.nx, y = ii / L.nx;
    const Co<T> k = coef_at<T>(L, i, x, y);
    const T om = static_cast<T>(kOmega);
    for (int q = 0; q < nv; q += 2) {
        const bool two = q + 1 < nv;
        const St<T> u0 = stencil(k, v.in[q], i, L.nx);
        const T b0 = v.b[q][i];
        St<T> u1{};
        T b1 = T(0);
        if (two) {
            u1 = stencil(k, v.in[q + 1], i, L.nx);
            b1 = v.b[q + 1][i];
        }
        const T c0 = static_cast<T>(v.c[q]);
        const T r0 = b0 - apply_st(k, u0, c0);
        v.out[q][i] = SWEEP ? u0.c + om * r0 / (k.d - c0) : r0;
        if (two) {
            const T c1 = static_cast<T>(v.c[q + 1]);
            const T r1 = b1 - apply_st(k, u1, c1);
            v.out[q + 1][i] = SWEEP ? u1.c + om * r1 / (k.d - c1) : r1;
        }
    }
}

// Two sweeps from zero: u1 = omega b / (d - c) at every point, out = u1 + omega (b -
// (A - cI) u1) / (d - c); u1 at the neighbours is formed from their b and diagonal.
template <typename T>
__global__ void sweep2_from_zero_kernel(const MgLevel L, const MgVecsT<T> v, int nv) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int ii = static_cast<int>(i), x = ii % L.nx, y = ii / L.nx;
    const Co<T> k = coef_at<T>(L, i, x, y);
    const St<T> dg = stencil(k, diag_of<T>(L), i, L.nx);
    const T om = static_cast<T>(kOmega);
    auto first = [&](const St<T>& b, T c) {
        St<T> u;
        u.c = om * b.c / (dg.c - c);
        u.e = k.he ? om * b.e / (dg.e - c) : T(0);
        u.w = k.hw ? om * b.w / (dg.w - c) : T(0);
        u.n = k.hn ? om * b.n / (dg.n - c) : T(0);
        u.s = k.hs ? om * b.s / (dg.s - c) : T(0);
        return u;
    };
    for (int q = 0; q < nv; q += 2) {
        const bool two = q + 1 < nv;
        const St<T> b0 = stencil(k, v.b[q], i, L.nx);
        St<T> b1{};
        if (two) b1 = stencil(k, v.b[q + 1], i, L.nx);
        const T c0 = static_cast<T>(v.c[q]);
        const St<T> u0 = first(b0, c0);
        v.out[q][i] = u0.c + om * (b0.c - apply_st(k, u0, c0)) / (k.d - c0);
        if (two) {
            const T c1 = static_cast<T>(v.c[q + 1]);
            const St<T> u1 = first(b1, c1);
            v.out[q + 1][i] = u1.c + om * (b1.c - apply_st(k, u1, c1)) / (k.d - c1);
        }
    }
}

// Linear interpolation of fine index x from a coarse line of nc points (coarsened) or
// the identity, as two (index, weight) pairs; an absent entry has weight 0 and a valid
// (clamped) index, so the 2 x 2 sum below needs no branches or private arrays.
struct Interp {
    int j0, j1;
    double w0, w1;
};
__device__ __forceinline__ Interp interp(int x, int nc, int coarsened) {
    Interp t;
    if (!coarsened) {
        t.j0 = t.j1 = x;
        t.w0 = 1.0;
        t.w1 = 0.0;
    } else if (x & 1) {
        t.j0 = t.j1 = (x - 1) >> 1;
        t.w0 = 1.0;
        t.w1 = 0.0;
    } else {
        const int lo = (x >> 1) - 1, hi = x >> 1;
        t.j0 = lo >= 0 ? lo : 0;
        t.w0 = lo >= 0 ? 0.5 : 0.0;
        t.j1 = hi < nc ? hi : nc - 1;
        t.w1 = hi < nc ? 0.5 : 0.0;
    }
    return t;
}

// fine out += P coarse in; grid (point blocks, vectors)
template <typename T>
__global__ void prolong_add_kernel(const MgLevel F, const MgLevel C, const MgVecsT<T> v) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= F.n) return;
    const int q = blockIdx.y;
    const int ii = static_cast<int>(i), x = ii % F.nx, y = ii / F.nx;
    const Interp ix = interp(x, C.nx, C.cx), iy = interp(y, C.ny, C.cy);
    const T* __restrict__ e = v.in[q];
    const T* __restrict__ r0 = e + iy.j0 * C.nx;
    const T* __restrict__ r1 = e + iy.j1 * C.nx;
    const T wx0 = static_cast<T>(ix.w0), wx1 = static_cast<T>(ix.w1);
    const T acc = static_cast<T>(iy.w0) * (wx0 * r0[ix.j0] + wx1 * r0[ix.j1]) +
                  static_cast<T>(iy.w1) * (wx0 * r1[ix.j0] + wx1 * r1[ix.j1]);
    v.out[q][i] += acc;
}

// coarse out = R fine in: per coarsened dimension fine 2J (1/2), 2J+1 (1), 2J+2 (1/2),
// divided by 2 per coarsened dimension; grid (point blocks, vectors)
template <typename T>
__global__ void restrict_kernel(const MgLevel F, const MgLevel C, const MgVecsT<T> v) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= C.n) return;
    const int q = blockIdx.y;
    const int ii = static_cast<int>(i), X = ii % C.nx, Y = ii / C.nx;
    const T* __restrict__ in = v.in[q];
    const T wd[3] = {T(0.5), T(1), T(0.5)};
    T acc = T(0);
    for (int dy = 0; dy < (C.cy ? 3 : 1); ++dy) {
        const int y = C.cy ? 2 * Y + dy : Y;
        if (y >= F.ny) continue;
        const T wy = C.cy ? wd[dy] : T(1);
        for (int dx = 0; dx < (C.cx ? 3 : 1); ++dx) {
            const int x = C.cx ? 2 * X + dx : X;
            if (x >= F.nx) continue;
            const T wx = C.cx ? wd[dx] : T(1);
            acc += wy * wx * in[static_cast<long long>(y) * F.nx + x];
        }
    }
    v.out[q][i] = acc / static_cast<T>(1 << (C.cx + C.cy));
}

// ---- the coarse tail of the cycle in one kernel ------------------------------------
// Levels of at most kTailN points cost a few microseconds per launch whatever their
// size, so the part of the cycle from the first such level down to the coarsest and back
// up runs in one kernel: one workgroup per vector, each phase a strided loop over the
// level's points followed by a workgroup barrier (which orders the phases' global
// writes and reads).  Same arithmetic as the per-level kernels.
constexpr long long kTailN = 4096;
constexpr int kTailMax = 13;  // levels from 4096 points down to at most 4 (1D: 11)
constexpr int kTailThreads = 256;

template <typename T>
struct TailArgs {
    int lt, nl;                  // first tail level, number of tail levels
    MgLevel lev[kTailMax + 1];   // lev[0]: the level above the tail (unused when lt == 0)
    const T* b0[kMgMaxVec];      // right-hand sides of the first tail level
    T* r0[kMgMaxVec];            // its results
    T* u0[kMgMaxVec];            // its work vectors
    T* base[kTailMax];           // levels below the first: B | U | R blocks of nv vectors
    double c[kMgMaxVec];
    int nv;
};

template <typename T>
__device__ void tail_sweep2(const MgLevel& L, const T* __restrict__ b, T* __restrict__ o, T c) {
    const T om = static_cast<T>(kOmega);
    const T* dgp = diag_of<T>(L);
    for (long long i = threadIdx.x; i < L.n; i += blockDim.x) {
        const int ii = static_cast<int>(i), x = ii % L.nx, y = ii / L.nx;
        const Co<T> k = coef_at<T>(L, i, x, y);
        const St<T> dg = stencil(k, dgp, i, L.nx);
        const St<T> bb = stencil(k, b, i, L.nx);
        St<T> u;
        u.c = om * bb.c / (dg.c - c);
        u.e = k.he ? om * bb.e / (dg.e - c) : T(0);
        u.w = k.hw ? om * bb.w / (dg.w - c) : T(0);
        u.n = k.hn ? om * bb.n / (dg.n - c) : T(0);
        u.s = k.hs ? om * bb.s / (dg.s - c) : T(0);
        o[i] = u.c + om * (bb.c - apply_st(k, u, c)) / (k.d - c);
    }
}
template <typename T, bool SWEEP>
__device__ void tail_sweep(const MgLevel& L, const T* __restrict__ u, const T* __restrict__ b, T* __restrict__ o,
                           T c) {
    const T om = static_cast<T>(kOmega);
    for (long long i = threadIdx.x; i < L.n; i += blockDim.x) {
        const int ii = static_cast<int>(i), x = ii % L.nx, y = ii / L.nx;
        const Co<T> k = coef_at<T>(L, i, x, y);
        const St<T> uu = stencil(k, u, i, L.nx);
        const T r = b[i] - apply_st(k, uu, c);
        o[i] = SWEEP ? uu.c + om * r / (k.d - c) : r;
    }
}
template <typename T>
__device__ void tail_restrict(const MgLevel& F, const MgLevel& C, const T* __restrict__ in, T* __restrict__ o) {
    const T wd[3] = {T(0.5), T(1), T(0.5)};
    for (long long i = threadIdx.x; i < C.n; i += blockDim.x) {
        const int ii = static_cast<int>(i), X = ii % C.nx, Y = ii / C.nx;
        T acc = T(0);
        for (int dy = 0; dy < (C.cy ? 3 : 1); ++dy) {
            const int y = C.cy ? 2 * Y + dy : Y;
            if (y >= F.ny) continue;
            const T wy = C.cy ? wd[dy] : T(1);
            for (int dx = 0; dx < (C.cx ? 3 : 1); ++dx) {
                const int x = C.cx ? 2 * X + dx : X;
                if (x >= F.nx) continue;
                const T wx = C.cx ? wd[dx] : T(1);
                acc += wy * wx * in[static_cast<long long>(y) * F.nx + x];
            }
        }
        o[i] = acc / static_cast<T>(1 << (C.cx + C.cy));
    }
}
template <typename T>
__device__ void tail_prolong_add(const MgLevel& F, const MgLevel& C, const T* __restrict__ e, T* __restrict__ o) {
    for (long long i = threadIdx.x; i < F.n; i += blockDim.x) {
        const int ii = static_cast<int>(i), x = ii % F.nx, y = ii / F.nx;
        const Interp ix = interp(x, C.nx, C.cx), iy = interp(y, C.ny, C.cy);
        const T* r0 = e + iy.j0 * C.nx;
        const T* r1 = e + iy.j1 * C.nx;
        const T wx0 = static_cast<T>(ix.w0), wx1 = static_cast<T>(ix.w1);
        o[i] += static_cast<T>(iy.w0) * (wx0 * r0[ix.j0] + wx1 * r0[ix.j1]) +
                static_cast<T>(iy.w1) * (wx0 * r1[ix.j0] + wx1 * r1[ix.j1]);
    }
}
template <typename T>
__device__ void tail_coarsest(const MgLevel& L, const T* __restrict__ b, T* __restrict__ o, double c) {
    if (threadIdx.x != 0) return;
    const int n = static_cast<int>(L.n);
    double M[4][4], r[4];
    for (int a = 0; a < n; ++a) {
        for (int bb = 0; bb < n; ++bb) M[a][bb] = 0.0;
        r[a] = static_cast<double>(b[a]);
    }
    for (int a = 0; a < n; ++a) {
        const int x = a % L.nx, y = a / L.nx;
        M[a][a] = L.diag[a] - c;
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
            for (int bb = k; bb < n; ++bb) M[a][bb] -= f * M[k][bb];
            r[a] -= f * r[k];
        }
    for (int a = n - 1; a >= 0; --a) {
        double t = r[a];
        for (int bb = a + 1; bb < n; ++bb) t -= M[a][bb] * r[bb];
        r[a] = t / M[a][a];
    }
    for (int a = 0; a < n; ++a) o[a] = static_cast<T>(r[a]);
}

// One workgroup per vector q: the V-cycle from tail level 0 (= hierarchy level lt) down
// and back up; the result lands in r0[q].
template <typename T>
__global__ __launch_bounds__(kTailThreads) void tail_kernel(const TailArgs<T> a) {
    const int q = blockIdx.x;
    const T c = static_cast<T>(a.c[q]);
    const MgLevel* lv = a.lev + 1;  // lv[k] = hierarchy level lt + k
    auto B = [&](int k) -> T* { return k == 0 ? const_cast<T*>(a.b0[q]) : a.base[k] + static_cast<long long>(q) * lv[k].n; };
    auto U = [&](int k) -> T* {
        return k == 0 ? a.u0[q] : a.base[k] + static_cast<long long>(a.nv + q) * lv[k].n;
    };
    auto R = [&](int k) -> T* {
        return k == 0 ? a.r0[q] : a.base[k] + static_cast<long long>(2 * a.nv + q) * lv[k].n;
    };
    const int last = a.nl - 1;
    for (int k = 0; k < last; ++k) {
        tail_sweep2(lv[k], B(k), R(k), c);
        __syncthreads();
        tail_sweep<T, false>(lv[k], R(k), B(k), U(k), c);
        __syncthreads();
        tail_restrict(lv[k], lv[k + 1], U(k), B(k + 1));
        __syncthreads();
    }
    tail_coarsest(lv[last], B(last), R(last), a.c[q]);
    __syncthreads();
    for (int k = last - 1; k >= 0; --k) {
        tail_prolong_add(lv[k], lv[k + 1], R(k + 1), R(k));
        __syncthreads();
        tail_sweep<T, true>(lv[k], R(k), B(k), U(k), c);
        __syncthreads();
        tail_sweep<T, true>(lv[k], U(k), B(k), R(k), c);
        __syncthreads();
    }
}

// float32 copies of a level's diagonal and face arrays
__global__ void to_float_kernel(const MgLevel L) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    L.diag_f[i] = static_cast<float>(L.diag[i]);
    L.wx_f[i] = static_cast<float>(L.wx[i]);
    L.wy_f[i] = static_cast<float>(L.wy[i]);
}

template <typename T>
hipError_t vcycle_t(const MgHierarchy& h, int nv, const T* const* b, T* const* u, const double* c, T* scratch,
                    hipStream_t s) {
    if (nv < 1 || nv > kMgMaxVec || h.nlev < 1) return hipErrorInvalidValue;
    // per level: B (right-hand sides), U (work), T (result)
    const T* B[kMgMaxLevels][kMgMaxVec];
    T* U[kMgMaxLevels][kMgMaxVec];
    T* R[kMgMaxLevels][kMgMaxVec];
    T* p = scratch;
    for (int q = 0; q < nv; ++q) {
        B[0][q] = b[q];
        R[0][q] = u[q];
        U[0][q] = p + static_cast<size_t>(q) * h.lev[0].n;
    }
    p += static_cast<size_t>(nv) * h.lev[0].n;
    for (int l = 1; l < h.nlev; ++l) {
        const size_t n = h.lev[l].n;
        for (int q = 0; q < nv; ++q) {
            B[l][q] = p + q * n;
            U[l][q] = p + (nv + q) * n;
            R[l][q] = p + (2 * nv + q) * n;
        }
        p += 3 * nv * n;
    }
    auto vecs = [&](T* const* in, const T* const* rhs, T* const* out) {
        MgVecsT<T> v{};
        for (int q = 0; q < nv; ++q) {
            v.in[q] = in ? in[q] : nullptr;
            v.b[q] = rhs ? rhs[q] : nullptr;
            v.out[q] = out[q];
            v.c[q] = c[q];
        }
        return v;
    };
    // the first level of the fused coarse tail
    int lt = 0;
    while (lt < h.nlev - 1 && h.lev[lt].n > kTailN) ++lt;
    if (h.nlev - lt > kTailMax) return hipErrorInvalidValue;
    // down the hierarchy to the tail: two sweeps from zero, residual, restriction
    for (int l = 0; l < lt; ++l) {
        const MgLevel& L = h.lev[l];
        const dim3 g(grid_of(L.n));
        hipLaunchKernelGGL(sweep2_from_zero_kernel<T>, g, dim3(256), 0, s, L, vecs(nullptr, B[l], R[l]), nv);
        hipLaunchKernelGGL((sweep_kernel<T, false>), g, dim3(256), 0, s, L, vecs(R[l], B[l], U[l]), nv);
        T* const* Bn = const_cast<T* const*>(B[l + 1]);
        hipLaunchKernelGGL(restrict_kernel<T>, dim3(grid_of(h.lev[l + 1].n), nv), dim3(256), 0, s, L, h.lev[l + 1],
                           vecs(U[l], nullptr, Bn));
    }
    // the tail: levels lt .. nlev-1 in one kernel, one workgroup per vector
    {
        TailArgs<T> ta{};
        ta.lt = lt;
        ta.nl = h.nlev - lt;
        ta.nv = nv;
        for (int k = 0; k < ta.nl; ++k) ta.lev[k + 1] = h.lev[lt + k];
        for (int q = 0; q < nv; ++q) {
            ta.b0[q] = B[lt][q];
            ta.r0[q] = R[lt][q];
            ta.u0[q] = U[lt][q];
            ta.c[q] = c[q];
        }
        // levels below lt keep the B | U | R layout of the scratch (base = B of vector 0)
        for (int k = 1; k < ta.nl; ++k) ta.base[k] = const_cast<T*>(B[lt + k][0]);
        hipLaunchKernelGGL(tail_kernel<T>, dim3(nv), dim3(kTailThreads), 0, s, ta);
    }
    // and back up from the tail: correction, two sweeps
    for (int l = lt - 1; l >= 0; --l) {
        const MgLevel& L = h.lev[l];
        const dim3 g(grid_of(L.n));
        hipLaunchKernelGGL(prolong_add_kernel<T>, dim3(grid_of(L.n), nv), dim3(256), 0, s, L, h.lev[l + 1],
                           vecs(R[l + 1], nullptr, R[l]));
        hipLaunchKernelGGL((sweep_kernel<T, true>), g, dim3(256), 0, s, L, vecs(R[l], B[l], U[l]), nv);
        hipLaunchKernelGGL((sweep_kernel<T, true>), g, dim3(256), 0, s, L, vecs(U[l], B[l], R[l]), nv);
    }
    return hipGetLastError();
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
    // float64 diagonal and faces, Dirichlet faces, and the float32 copies (3n floats)
    return 3 * static_cast<size_t>(L.n) + 2 * static_cast<size_t>(L.nx) + 2 * static_cast<size_t>(L.ny) +
           (3 * static_cast<size_t>(L.n) + 1) / 2;
}

hipError_t mg_build(const MgHierarchy& h, const double* kappa, hipStream_t s) {
    hipLaunchKernelGGL(fine_faces_kernel, dim3(grid_of(h.lev[0].n)), dim3(256), 0, s, h.lev[0], kappa);
    hipLaunchKernelGGL(diag_kernel, dim3(grid_of(h.lev[0].n)), dim3(256), 0, s, h.lev[0]);
    for (int l = 1; l < h.nlev; ++l) {
        hipLaunchKernelGGL(coarsen_faces_kernel, dim3(grid_of(h.lev[l].n)), dim3(256), 0, s, h.lev[l - 1], h.lev[l]);
        hipLaunchKernelGGL(diag_kernel, dim3(grid_of(h.lev[l].n)), dim3(256), 0, s, h.lev[l]);
    }
    for (int l = 0; l < h.nlev; ++l)
        hipLaunchKernelGGL(to_float_kernel, dim3(grid_of(h.lev[l].n)), dim3(256), 0, s, h.lev[l]);
    return hipGetLastError();
}

size_t mg_scratch_elems(const MgHierarchy& h, int nv) {
    // level 0: one work vector per right-hand side; coarser levels: b, u, t
    size_t d = static_cast<size_t>(nv) * h.lev[0].n;
    for (int l = 1; l < h.nlev; ++l) d += 3 * static_cast<size_t>(nv) * h.lev[l].n;
    return d;
}

hipError_t mg_vcycle(const MgHierarchy& h, int nv, const double* const* b, double* const* u, const double* c,
                     double* scratch, hipStream_t s) {
    return vcycle_t<double>(h, nv, b, u, c, scratch, s);
}

hipError_t mg_vcycle(const MgHierarchy& h, int nv, const float* const* b, float* const* u, const double* c,
                     float* scratch, hipStream_t s) {
    return vcycle_t<float>(h, nv, b, u, c, scratch, s);
}

}  // namespace ac
