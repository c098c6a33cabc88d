// Exact shifted solves for a constant coefficient on a Dirichlet grid (Appendix A).
// There A = I + kappa (T_x (+) T_y) with T = tridiag(-1, 2, -1), and the orthonormal
// DST-I matrix S_x (symmetric, its own inverse) diagonalises T_x with eigenvalues
// mu_k = 4 sin^2(k pi / (2 (n_x + 1))), k = 1..n_x.  After r -> S_x r along x, mode
// k of (A - lambda I) y = r is the tridiagonal system along y
//   (1 + kappa (mu_k + 2) - lambda) y_j - kappa (y_{j-1} + y_{j+1}) = r_j
// (one dimension: the scalar (1 + kappa mu_k - lambda) y = r), strictly diagonally
// dominant since Re lambda <= |lambda| = alpha^{1/l} <= 1, so elimination without
// pivoting is stable.  Then y = S_x (solution).
//
// S_x has the reflection symmetry S[k][n-1-i] = (-1)^k S[k][i], so one butterfly level
// halves each transform: the even modes k = 2m see only u_i = x_i + x_{n-1-i} (and the
// middle point for odd n), the odd modes k = 2m+1 only v_i = x_i - x_{n-1-i}, each a
// dense product with a half-size block of S_x (matrix-core GEMMs, exact_gemm.hip).
// Spectral data are kept in that order (h = ceil(n_x/2) even modes, then n_x - h odd
// modes); the inverse
// transform ends with x_i = E_i + O_i, x_{n-1-i} = E_i - O_i.  This file holds the half
// matrices, the split into planes fused with the butterfly, the merge fused with its
// inverse, and the tridiagonal solves, run as chunked scans over y so that every
// x mode and slot spreads over many threads.
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr double kPiE = 3.14159265358979323846;

__device__ __forceinline__ double dst_entry(long long k, long long i, int n) {
    // sqrt(2/(n+1)) sin((k+1)(i+1) pi / (n+1)), the angle's multiple of pi/(n+1)
    // reduced modulo 2 (n+1) first
    const long long m = ((k + 1) * (i + 1)) % (2LL * (n + 1));
    return sqrt(2.0 / (n + 1)) * sin(kPiE * static_cast<double>(m) / (n + 1));
}

// Half matrices, column-major: Se (h x h), Se(m, i) = S[2m][i]; So (h2 x h2),
// So(m, i) = S[2m+1][i]; h = ceil(n/2), h2 = floor(n/2).  So starts h*h entries in.
template <typename R>
__global__ void dst_half_kernel(R* __restrict__ S, int n) {
    const long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long long h = (n + 1) / 2, h2 = n / 2;
    if (q < h * h) {
        const long long m = q % h, i = q / h;
        S[q] = static_cast<R>(dst_entry(2 * m, i, n));
    } else if (q < h * h + h2 * h2) {
        const long long r = q - h * h, m = r % h2, i = r / h2;
        S[q] = static_cast<R>(dst_entry(2 * m + 1, i, n));
    }
}

// Thread (x < h, row y, slot): SPLIT reads x and its mirror n-1-x of grid row y and
// writes u (row x) and v (row h + x) of the row's plane column; otherwise reads E
// (row x) and O (row h + x) and writes E + O and E - O back to the two grid points.
template <typename R, bool SPLIT>
__device__ __forceinline__ void butterfly(R* __restrict__ z, int zs, R* __restrict__ col, int nx, int x) {
    const int h = (nx + 1) / 2, h2 = nx / 2;
    const int xm = nx - 1 - x;
    if (SPLIT) {
        const R a = z[static_cast<long long>(x) * zs];
        if (x < h2) {
            const R b = z[static_cast<long long>(xm) * zs];
            col[x] = a + b;
            col[h + x] = a - b;
        } else {
            col[x] = a;  // middle point of odd n
        }
    } else {
        const R e = col[x];
        if (x < h2) {
            const R o = col[h + x];
            z[static_cast<long long>(x) * zs] = e + o;
            z[static_cast<long long>(xm) * zs] = e - o;
        } else {
            z[static_cast<long long>(x) * zs] = e;
        }
    }
}

// grid (ceil(h/64), ny, slots), 64 threads
template <typename R, bool SPLIT>
__global__ __launch_bounds__(64) void planes_kernel(const ExactArgs a, R* __restrict__ planes) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, s = blockIdx.z;
    if (x >= (a.nx + 1) / 2) return;
    const long long row = static_cast<long long>(y) * a.nx;
    R* col = planes + static_cast<long long>(a.plane[s]) * a.n + row;
    R* z = static_cast<R*>(a.slot[s]);
    if (a.cplx[s]) {
        butterfly<R, SPLIT>(z + 2 * row, 2, col, a.nx, x);
        butterfly<R, SPLIT>(z + 2 * row + 1, 2, col + a.n, a.nx, x);
    } else {
        butterfly<R, SPLIT>(z + row, 1, col, a.nx, x);
    }
}

struct cd {
    double r, i;
};
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.r * s, a.i * s}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
__device__ __forceinline__ cd csqrt_(cd z) {
    const double m = hypot(z.r, z.i);
    const double re = sqrt(fmax(0.5 * (m + z.r), 0.0));
    const double im = copysign(sqrt(fmax(0.5 * (m - z.r), 0.0)), z.i);
    return {re, im};
}
// t^n for n >= 1
__device__ __forceinline__ cd cpow_(cd t, int n) {
    if (t.r == 0.0 && t.i == 0.0) return {0.0, 0.0};
    const double lm = 0.5 * log(t.r * t.r + t.i * t.i), th = atan2(t.i, t.r);
    const double mag = exp(n * lm);
    double sn, cs;
    sincos(n * th, &sn, &cs);
    return {mag * cs, mag * sn};
}

// Rows per chunk of the scan over y (a chunk's rows stay in registers).
constexpr int kC = 16;

// Column (x mode k, slot s) of the tridiagonal system along y: diagonal b, off-diagonal
// e.  Elimination without pivoting has pivots den_j = D_{j+1}/D_j, D_j the leading
// principal minors, D_{j+1} = b D_j - e^2 D_{j-1}; with r1, r2 the roots of
// r^2 - b r + e^2 = 0, |r1| >= |r2| (strictly, by diagonal dominance), and t = r2/r1,
//   den_j = r1 (1 - t^{j+2}) / (1 - t^{j+1}),
// so every row's pivot is known without the sequential recurrence.  With h_j = -e/den_j
// the forward sweep is f_j = d_j/den_j + h_j f_{j-1} and the back substitution
// y_j = f_j + h_j y_{j+1}: both linear first-order recurrences with |h_j| < 1, solved
// chunk-wise (local sweeps from zero, then the carries between chunks).
struct Column {
    cd r1, t;
    double e;
};

// r: spectral row (even modes first), mode k = 2r or 2(r - h) + 1
__device__ Column column_of(const ExactArgs& a, int r, int s) {
    const int h = (a.nx + 1) / 2;
    const int k = r < h ? 2 * r : 2 * (r - h) + 1;
    const double sk = sin(kPiE * (k + 1) / (2.0 * (a.nx + 1)));
    const bool two = a.dim == 2;
    const cd b = {1.0 + a.kappa * (4.0 * sk * sk + (two ? 2.0 : 0.0)) - a.lr[s], -a.li[s]};
    Column c;
    c.e = two ? -a.kappa : 0.0;
    if (c.e == 0.0) {
        c.r1 = b;
        c.t = {0.0, 0.0};
        return c;
    }
    const cd sq = csqrt_(cadd(cmul(b, b), {-4.0 * c.e * c.e, 0.0}));
    const cd p = cscale(cadd(b, sq), 0.5), m = cscale(cadd(b, cscale(sq, -1.0)), 0.5);
    c.r1 = (p.r * p.r + p.i * p.i >= m.r * m.r + m.i * m.i) ? p : m;
    const cd r2 = cdiv({c.e * c.e, 0.0}, c.r1);
    c.t = cdiv(r2, c.r1);
    return c;
}

// 1/den_j and h_j from tp1 = t^{j+1}; advances tp1 to t^{j+2}
__device__ __forceinline__ void row_coef(const Column& c, cd& tp1, cd& inv, cd& h) {
    const cd tp2 = cmul(tp1, c.t);
    inv = cdiv({1.0 - tp1.r, -tp1.i}, cmul(c.r1, {1.0 - tp2.r, -tp2.i}));
    h = cscale(inv, -c.e);
    tp1 = tp2;
}

template <typename R, bool CPLX>
__device__ __forceinline__ cd load_c(const R* re, long long o, long long n) {
    return {static_cast<double>(re[o]), CPLX ? static_cast<double>(re[o + n]) : 0.0};
}
template <typename R, bool CPLX>
__device__ __forceinline__ void store_c(R* re, long long o, long long n, cd v) {
    re[o] = static_cast<R>(v.r);
    if (CPLX) re[o + n] = static_cast<R>(v.i);
}

struct ScanGeom {
    int k, s, q, y0, rows;
    long long pl;   // first element of the slot's real plane
    long long cix;  // carry index (s, q, k)
};

__device__ __forceinline__ bool scan_geom(const ExactArgs& a, int nq, ScanGeom& g) {
    g.k = blockIdx.x * blockDim.x + threadIdx.x;
    g.q = blockIdx.y;
    g.s = blockIdx.z;
    if (g.k >= a.nx) return false;
    g.y0 = g.q * kC;
    g.rows = min(kC, a.ny - g.y0);
    g.pl = static_cast<long long>(a.plane[g.s]) * a.n;
    g.cix = (static_cast<long long>(g.s) * nq + g.q) * a.nx + g.k;
    return true;
}

// Forward sweep of one chunk from a zero carry: u_j = d_j/den_j + h_j u_{j-1}.
// fl = last u of the chunk, hp = product of the chunk's h_j.
template <typename R, bool CPLX>
__device__ __forceinline__ void fwd_local(const ExactArgs& a, const ScanGeom& g, const R* __restrict__ d, R* __restrict__ u,
                          cd* __restrict__ fl, cd* __restrict__ hp) {
    const Column c = column_of(a, g.k, g.s);
    cd v[kC];
#pragma unroll
    for (int j = 0; j < kC; ++j)
        v[j] = j < g.rows ? load_c<R, CPLX>(d + g.pl, static_cast<long long>(g.y0 + j) * a.nx + g.k, a.n) : cd{0.0, 0.0};
    cd tp1 = cpow_(c.t, g.y0 + 1), acc = {0.0, 0.0}, prod = {1.0, 0.0};
#pragma unroll
    for (int j = 0; j < kC; ++j) {
        if (j < g.rows) {
            cd inv, h;
            row_coef(c, tp1, inv, h);
            acc = cadd(cmul(v[j], inv), cmul(h, acc));
            prod = cmul(prod, h);
            store_c<R, CPLX>(u + g.pl, static_cast<long long>(g.y0 + j) * a.nx + g.k, a.n, acc);
        }
    }
    fl[g.cix] = acc;
    hp[g.cix] = prod;
}

// Forward fix-up with the carry-in f_{y0-1} (din), then the backward sweep of the chunk
// from a zero right carry: x_j = f_j + h_j x_{j+1}.  x0 = the chunk's first x.
template <typename R, bool CPLX>
__device__ __forceinline__ void bwd_local(const ExactArgs& a, const ScanGeom& g, const R* __restrict__ u, R* __restrict__ xp,
                          const cd* __restrict__ din, cd* __restrict__ x0) {
    const Column c = column_of(a, g.k, g.s);
    cd f[kC], h[kC];
#pragma unroll
    for (int j = 0; j < kC; ++j)
        f[j] = j < g.rows ? load_c<R, CPLX>(u + g.pl, static_cast<long long>(g.y0 + j) * a.nx + g.k, a.n) : cd{0.0, 0.0};
    const cd carry = din[g.cix];
    cd tp1 = cpow_(c.t, g.y0 + 1), prod = {1.0, 0.0};
#pragma unroll
    for (int j = 0; j < kC; ++j) {
        cd inv;
        row_coef(c, tp1, inv, h[j]);
        prod = cmul(prod, h[j]);
        f[j] = cadd(f[j], cmul(prod, carry));
    }
    cd x = {0.0, 0.0};
#pragma unroll
    for (int j = kC - 1; j >= 0; --j) {
        if (j < g.rows) {
            x = cadd(f[j], cmul(h[j], x));
            store_c<R, CPLX>(xp + g.pl, static_cast<long long>(g.y0 + j) * a.nx + g.k, a.n, x);
        }
    }
    x0[g.cix] = x;
}

// Backward fix-up with the right carry x_{y1} (xin): x_j += (h_j ... h_{y1-1}) xin.
template <typename R, bool CPLX>
__device__ __forceinline__ void bwd_fix(const ExactArgs& a, const ScanGeom& g, const R* __restrict__ xp, R* __restrict__ x,
                        const cd* __restrict__ xin) {
    const Column c = column_of(a, g.k, g.s);
    cd v[kC], h[kC];
#pragma unroll
    for (int j = 0; j < kC; ++j)
        v[j] = j < g.rows ? load_c<R, CPLX>(xp + g.pl, static_cast<long long>(g.y0 + j) * a.nx + g.k, a.n) : cd{0.0, 0.0};
    const cd carry = xin[g.cix];
    cd tp1 = cpow_(c.t, g.y0 + 1);
#pragma unroll
    for (int j = 0; j < kC; ++j) {
        cd inv;
        row_coef(c, tp1, inv, h[j]);
    }
    cd prod = {1.0, 0.0};
#pragma unroll
    for (int j = kC - 1; j >= 0; --j) {
        if (j < g.rows) {
            prod = cmul(prod, h[j]);
            store_c<R, CPLX>(x + g.pl, static_cast<long long>(g.y0 + j) * a.nx + g.k, a.n,
                             cadd(v[j], cmul(prod, carry)));
        }
    }
}

// grid (ceil(nx/64), chunks, slots), 64 threads
template <typename R>
__global__ __launch_bounds__(64) void fwd_local_kernel(const ExactArgs a, int nq, const R* __restrict__ d,
                                                       R* __restrict__ u, cd* __restrict__ fl, cd* __restrict__ hp) {
    ScanGeom g;
    if (!scan_geom(a, nq, g)) return;
    if (a.cplx[g.s]) fwd_local<R, true>(a, g, d, u, fl, hp);
    else fwd_local<R, false>(a, g, d, u, fl, hp);
}
template <typename R>
__global__ __launch_bounds__(64) void bwd_local_kernel(const ExactArgs a, int nq, const R* __restrict__ u,
                                                       R* __restrict__ xp, const cd* __restrict__ din,
                                                       cd* __restrict__ x0) {
    ScanGeom g;
    if (!scan_geom(a, nq, g)) return;
    if (a.cplx[g.s]) bwd_local<R, true>(a, g, u, xp, din, x0);
    else bwd_local<R, false>(a, g, u, xp, din, x0);
}
template <typename R>
__global__ __launch_bounds__(64) void bwd_fix_kernel(const ExactArgs a, int nq, const R* __restrict__ xp,
                                                     R* __restrict__ x, const cd* __restrict__ xin) {
    ScanGeom g;
    if (!scan_geom(a, nq, g)) return;
    if (a.cplx[g.s]) bwd_fix<R, true>(a, g, xp, x, xin);
    else bwd_fix<R, false>(a, g, xp, x, xin);
}

// Carries between chunks, one thread per (x mode, slot); grid (ceil(nx/64), slots).
// The loads of kB chunks are issued together ahead of their sequential combination.
constexpr int kB = 8;

// Forward: f_{end of q} = fl_q + hp_q f_{end of q-1}; fl_q is replaced by the carry-in.
__global__ __launch_bounds__(64) void fwd_carry_kernel(int nx, int nq, cd* __restrict__ fl, const cd* __restrict__ hp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nx) return;
    const long long base = static_cast<long long>(blockIdx.y) * nq * nx + k;
    cd f = {0.0, 0.0};
    for (int q0 = 0; q0 < nq; q0 += kB) {
        cd v[kB], m[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const long long o = base + static_cast<long long>(q0 + j) * nx;
            v[j] = q0 + j < nq ? fl[o] : cd{0.0, 0.0};
            m[j] = q0 + j < nq ? hp[o] : cd{0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            if (q0 + j < nq) {
                fl[base + static_cast<long long>(q0 + j) * nx] = f;
                f = cadd(v[j], cmul(m[j], f));
            }
        }
    }
}
// Backward: x_{start of q} = x0_q + hp_q x_{start of q+1}; x0_q is replaced by the
// right carry x_{start of q+1}.
__global__ __launch_bounds__(64) void bwd_carry_kernel(int nx, int nq, cd* __restrict__ x0, const cd* __restrict__ hp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nx) return;
    const long long base = static_cast<long long>(blockIdx.y) * nq * nx + k;
    cd x = {0.0, 0.0};
    for (int q1 = nq - 1; q1 >= 0; q1 -= kB) {
        cd v[kB], m[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const long long o = base + static_cast<long long>(q1 - j) * nx;
            v[j] = q1 - j >= 0 ? x0[o] : cd{0.0, 0.0};
            m[j] = q1 - j >= 0 ? hp[o] : cd{0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            if (q1 - j >= 0) {
                x0[base + static_cast<long long>(q1 - j) * nx] = x;
                x = cadd(v[j], cmul(m[j], x));
            }
        }
    }
}

int grid_of(long long n) { return static_cast<int>((n + 255) / 256); }

}  // namespace

long long dst_half_elems(int n) {
    const long long h = (n + 1) / 2, h2 = n / 2;
    return h * h + h2 * h2;
}

hipError_t launch_dst_half(int prec, void* S, int n, hipStream_t s) {
    const long long nn = dst_half_elems(n);
    if (prec == 0) hipLaunchKernelGGL(dst_half_kernel<double>, dim3(grid_of(nn)), dim3(256), 0, s, static_cast<double*>(S), n);
    else hipLaunchKernelGGL(dst_half_kernel<float>, dim3(grid_of(nn)), dim3(256), 0, s, static_cast<float*>(S), n);
    return hipGetLastError();
}

hipError_t launch_exact_planes(int prec, bool split, const ExactArgs& a, void* planes, hipStream_t s) {
    if (a.ny > 65535) return hipErrorInvalidValue;
    const dim3 grid(((a.nx + 1) / 2 + 63) / 64, a.ny, a.nslot);
    if (prec == 0) {
        if (split) hipLaunchKernelGGL((planes_kernel<double, true>), grid, dim3(64), 0, s, a, static_cast<double*>(planes));
        else hipLaunchKernelGGL((planes_kernel<double, false>), grid, dim3(64), 0, s, a, static_cast<double*>(planes));
    } else {
        if (split) hipLaunchKernelGGL((planes_kernel<float, true>), grid, dim3(64), 0, s, a, static_cast<float*>(planes));
        else hipLaunchKernelGGL((planes_kernel<float, false>), grid, dim3(64), 0, s, a, static_cast<float*>(planes));
    }
    return hipGetLastError();
}

int exact_chunks(int ny) { return (ny + kC - 1) / kC; }

size_t exact_carry_bytes(int nx, int ny, int nslot) {
    return 3 * static_cast<size_t>(nslot) * exact_chunks(ny) * nx * sizeof(cd);
}

template <typename R>
static hipError_t tridiag_t(const ExactArgs& a, R* t, R* u, void* carry, hipStream_t s) {
    const int nq = exact_chunks(a.ny);
    const size_t per = static_cast<size_t>(a.nslot) * nq * a.nx;
    cd* c0 = static_cast<cd*>(carry);
    cd* hp = c0 + per;
    cd* c1 = hp + per;
    const dim3 grid((a.nx + 63) / 64, nq, a.nslot), cgrid((a.nx + 63) / 64, a.nslot);
    // t: right-hand sides -> (forward) u -> (backward, local) t -> (fix-up) u
    hipLaunchKernelGGL(fwd_local_kernel<R>, grid, dim3(64), 0, s, a, nq, t, u, c0, hp);
    hipLaunchKernelGGL(fwd_carry_kernel, cgrid, dim3(64), 0, s, a.nx, nq, c0, hp);
    hipLaunchKernelGGL(bwd_local_kernel<R>, grid, dim3(64), 0, s, a, nq, u, t, c0, c1);
    hipLaunchKernelGGL(bwd_carry_kernel, cgrid, dim3(64), 0, s, a.nx, nq, c1, hp);
    hipLaunchKernelGGL(bwd_fix_kernel<R>, grid, dim3(64), 0, s, a, nq, t, u, c1);
    return hipGetLastError();
}

hipError_t launch_exact_tridiag(int prec, const ExactArgs& a, void* t, void* u, void* carry, hipStream_t s) {
    if (a.ny > kC * 65535) return hipErrorInvalidValue;
    if (prec == 0) return tridiag_t<double>(a, static_cast<double*>(t), static_cast<double*>(u), carry, s);
    return tridiag_t<float>(a, static_cast<float*>(t), static_cast<float*>(u), carry, s);
}

}  // namespace ac
