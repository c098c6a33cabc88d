// Exact shifted solves for a constant coefficient on a Dirichlet grid (Appendix A).
// There A = I + kappa (T_x (+) T_y) with T = tridiag(-1, 2, -1), and the orthonormal
// DST-I matrix S_x (symmetric, its own inverse) diagonalises T_x with eigenvalues
// mu_k = 4 sin^2(k pi / (2 (n_x + 1))), k = 1..n_x.  After r -> S_x r along x, mode
// k of (A - lambda I) y = r is the tridiagonal system along y
//   (1 + kappa (mu_k + 2) - lambda) y_j - kappa (y_{j-1} + y_{j+1}) = r_j
// (one dimension: the scalar (1 + kappa mu_k - lambda) y = r), strictly diagonally
// dominant since Re lambda <= |lambda| = alpha^{1/l} <= 1, so elimination without
// pivoting is stable.  Then y = S_x (solution).  The two dense transforms are
// library GEMMs; this file holds the DST matrix, the planar split and merge, and the
// tridiagonal elimination.
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr double kPiE = 3.14159265358979323846;

// S[i][j] = sqrt(2/(n+1)) sin((i+1)(j+1) pi / (n+1)), i, j < n
template <typename R>
__global__ void dst_matrix_kernel(R* __restrict__ S, int n) {
    const long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= static_cast<long long>(n) * n) return;
    const long long i = q / n, j = q % n;
    // reduce the angle's multiple of pi / (n+1) modulo 2 (n+1) before the sine
    const long long m = ((i + 1) * (j + 1)) % (2LL * (n + 1));
    S[q] = static_cast<R>(sqrt(2.0 / (n + 1)) * sin(kPiE * static_cast<double>(m) / (n + 1)));
}

// blockIdx.y = slot
template <typename R, bool SPLIT>
__global__ void planes_kernel(const ExactArgs a, R* __restrict__ planes) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= a.n) return;
    R* z = static_cast<R*>(a.slot[s]);
    R* re = planes + static_cast<long long>(a.plane[s]) * a.n;
    if (a.cplx[s]) {
        R* im = re + a.n;
        if (SPLIT) {
            re[i] = z[2 * i];
            im[i] = z[2 * i + 1];
        } else {
            z[2 * i] = re[i];
            z[2 * i + 1] = im[i];
        }
    } else {
        if (SPLIT) re[i] = z[i];
        else z[i] = re[i];
    }
}

struct cd {
    double r, i;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

constexpr int kU = 8;  // rows loaded ahead of the elimination

// Thread = (x mode k, slot).  Forward elimination: c'_0 = e/b, d'_0 = d_0/b,
// den_j = b - e c'_{j-1}, c'_j = e/den_j, d'_j = (d_j - e d'_{j-1})/den_j with
// e = -kappa the off-diagonal; back substitution y_j = d'_j - c'_j y_{j+1}.
// t: input d (overwritten by c'), u: d' then y.  Rows are read kU at a time so the
// loads of a batch are in flight together.
template <typename R, bool CPLX>
__device__ void tridiag_body(const ExactArgs& a, int k, int s, R* __restrict__ t, R* __restrict__ u) {
    const long long pl = static_cast<long long>(a.plane[s]) * a.n;
    R* tr = t + pl;
    R* ti = CPLX ? tr + a.n : nullptr;
    R* ur = u + pl;
    R* ui = CPLX ? ur + a.n : nullptr;
    const double sk = sin(kPiE * (k + 1) / (2.0 * (a.nx + 1)));
    const bool two = a.dim == 2;
    const cd b = {1.0 + a.kappa * (4.0 * sk * sk + (two ? 2.0 : 0.0)) - a.lr[s], -a.li[s]};
    const double e = two ? -a.kappa : 0.0;
    const int ny = a.ny;
    cd cp = {0.0, 0.0}, dp = {0.0, 0.0};
    for (int y0 = 0; y0 < ny; y0 += kU) {
        double vr[kU], vi[kU];
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            const int y = y0 + q;
            vr[q] = y < ny ? static_cast<double>(tr[static_cast<long long>(y) * a.nx + k]) : 0.0;
            vi[q] = (CPLX && y < ny) ? static_cast<double>(ti[static_cast<long long>(y) * a.nx + k]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            const int y = y0 + q;
            if (y >= ny) break;
            const cd den = {b.r - e * cp.r, b.i - e * cp.i};
            const cd num = {vr[q] - e * dp.r, vi[q] - e * dp.i};
            if (CPLX) {
                cp = cdiv({e, 0.0}, den);
                dp = cdiv(num, den);
            } else {
                cp = {e / den.r, 0.0};
                dp = {num.r / den.r, 0.0};
            }
            const long long o = static_cast<long long>(y) * a.nx + k;
            tr[o] = static_cast<R>(cp.r);
            ur[o] = static_cast<R>(dp.r);
            if (CPLX) {
                ti[o] = static_cast<R>(cp.i);
                ui[o] = static_cast<R>(dp.i);
            }
        }
    }
    // back substitution from the last row (y_{ny} = 0); the last row's d' was
    // just written and is still in dp
    cd yn = {0.0, 0.0};
    for (int y1 = ny - 1; y1 >= 0; y1 -= kU) {
        double cr[kU], ci[kU], dr[kU], di[kU];
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            const int y = y1 - q;
            const long long o = static_cast<long long>(y) * a.nx + k;
            cr[q] = y >= 0 ? static_cast<double>(tr[o]) : 0.0;
            dr[q] = y >= 0 ? static_cast<double>(ur[o]) : 0.0;
            ci[q] = (CPLX && y >= 0) ? static_cast<double>(ti[o]) : 0.0;
            di[q] = (CPLX && y >= 0) ? static_cast<double>(ui[o]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            const int y = y1 - q;
            if (y < 0) break;
            const cd c = {cr[q], ci[q]};
            const cd m = cmul(c, yn);
            yn = {dr[q] - m.r, di[q] - m.i};
            const long long o = static_cast<long long>(y) * a.nx + k;
            ur[o] = static_cast<R>(yn.r);
            if (CPLX) ui[o] = static_cast<R>(yn.i);
        }
    }
}

// blockIdx.y = slot; real slots take the real-arithmetic variant
template <typename R>
__global__ __launch_bounds__(256) void tridiag_kernel(const ExactArgs a, R* __restrict__ t, R* __restrict__ u) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (k >= a.nx) return;
    if (a.cplx[s]) tridiag_body<R, true>(a, k, s, t, u);
    else tridiag_body<R, false>(a, k, s, t, u);
}

int grid_of(long long n) { return static_cast<int>((n + 255) / 256); }

}  // namespace

hipError_t launch_dst_matrix(int prec, void* S, int n, hipStream_t s) {
    const long long nn = static_cast<long long>(n) * n;
    if (prec == 0) hipLaunchKernelGGL(dst_matrix_kernel<double>, dim3(grid_of(nn)), dim3(256), 0, s, static_cast<double*>(S), n);
    else hipLaunchKernelGGL(dst_matrix_kernel<float>, dim3(grid_of(nn)), dim3(256), 0, s, static_cast<float*>(S), n);
    return hipGetLastError();
}

hipError_t launch_exact_planes(int prec, bool split, const ExactArgs& a, void* planes, hipStream_t s) {
    const dim3 grid(grid_of(a.n), a.nslot);
    if (prec == 0) {
        if (split) hipLaunchKernelGGL((planes_kernel<double, true>), grid, dim3(256), 0, s, a, static_cast<double*>(planes));
        else hipLaunchKernelGGL((planes_kernel<double, false>), grid, dim3(256), 0, s, a, static_cast<double*>(planes));
    } else {
        if (split) hipLaunchKernelGGL((planes_kernel<float, true>), grid, dim3(256), 0, s, a, static_cast<float*>(planes));
        else hipLaunchKernelGGL((planes_kernel<float, false>), grid, dim3(256), 0, s, a, static_cast<float*>(planes));
    }
    return hipGetLastError();
}

hipError_t launch_exact_tridiag(int prec, const ExactArgs& a, void* t, void* u, hipStream_t s) {
    const dim3 grid(grid_of(a.nx), a.nslot);
    if (prec == 0)
        hipLaunchKernelGGL(tridiag_kernel<double>, grid, dim3(256), 0, s, a, static_cast<double*>(t), static_cast<double*>(u));
    else
        hipLaunchKernelGGL(tridiag_kernel<float>, grid, dim3(256), 0, s, a, static_cast<float*>(t), static_cast<float*>(u));
    return hipGetLastError();
}

}  // namespace ac
