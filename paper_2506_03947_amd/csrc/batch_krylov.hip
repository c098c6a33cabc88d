// Device-resident FGMRES for many independent problems: the Arnoldi step of every live
// problem (multi-dot, the one-reduction modified Gram-Schmidt coefficients, multi-axpy
// with the new norm, the Givens update and the convergence test), the cycle's solution
// update and the restart test run without the host, so a whole FGMRES cycle of all
// problems is one captured graph.
//
// The arithmetic is the single-problem solve's (ac_solve): modified Gram-Schmidt in
// inverse compact WY form with unnormalised basis vectors and their scales, Givens
// rotations on the Hessenberg matrix, x += Z y by back substitution.  The vector
// kernels share their bodies with the single-problem kernels (krylov_body.h) and walk
// a work list of the live problems (worklist.h); the scalar kernels run one workgroup
// per problem with the small matrices staged in LDS.  Partial sums are reduced in a
// fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ac_internal.h"
#include "krylov_body.h"
#include "worklist.h"

namespace ac {
namespace {

using namespace kry;

constexpr int kMB = kMaxBasis - 1;  // largest restart length

__device__ __forceinline__ LiveBlocks prob_live_blocks(const BKProb* P, int nprob, const int* live) {
    return live_blocks(
        nprob, [&](int q) { return P[q].nblk; }, [&](int q) { return live[q] != 0; });
}

__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Fixed-order sum over b < n of src[b * stride] by the whole workgroup (result valid in
// every thread after the call).
__device__ __forceinline__ double block_sum_strided(const double* __restrict__ src, int n, int stride) {
    __shared__ double part[kThreads / kWave];
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += kThreads) s += src[static_cast<long long>(b) * stride];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_down(s, off, kWave);
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) t += part[w];
    __syncthreads();
    return t;
}

// Step j (nv = j + 1 basis vectors): partials of V_q . w (q < nv), w . w and
// V_q . V_{nv-1} (q < nv - 1) with w = V_nv, as the single solve's multi-dot.
// KIND: 0, 1 element-split with 4 / 8 vectors; 2, 3 vector-parallel with 4 / 8 per wave.
template <int KIND>
__global__ __launch_bounds__(kThreads) void bk_mdot_kernel(const BKProb* __restrict__ P, int nprob,
                                                           const int* __restrict__ live, int nv) {
    const LiveBlocks W = prob_live_blocks(P, nprob, live);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const BKProb& p = list_args<BKProb>(P, q);
        const double* w = p.v0 + static_cast<long long>(nv) * p.vstride;
        double* out = p.partial + static_cast<long long>(local) * kBKRed;
        if (KIND == 0) mdot_es_body<4, true>(p.v0, p.vstride, nv, w, p.len, out, local, nb);
        else if (KIND == 1) mdot_es_body<8, true>(p.v0, p.vstride, nv, w, p.len, out, local, nb);
        else if (KIND == 2) mdot_vp_body<4, true>(p.v0, p.vstride, nv, w, p.len, out, local, nb);
        else mdot_vp_body<8, true>(p.v0, p.vstride, nv, w, p.len, out, local, nb);
        __syncthreads();  // the element-split bodies reuse their LDS on the next block
    }
}

// Gram-Schmidt coefficients of step j, one workgroup per live problem: the dots from
// the partials; row j of L (scaled dots of the newest basis vector with the older
// ones); (I + L) h = scaled V^T w by forward substitution; H column j = h; axpy
// coefficients scale_i h_i.
__global__ __launch_bounds__(kThreads) void bk_arnoldi_kernel(const BKProb* __restrict__ P, BKState* S,
                                                              const int* __restrict__ live, int j, int m) {
    const int q = blockIdx.x;
    if (!live[q]) return;
    constexpr int NW = kThreads / kWave;
    __shared__ double part[NW][2 * kMB];
    __shared__ double red[2 * kMB];
    __shared__ double Ls[kMB * kMB];
    const BKProb& p = list_args<BKProb>(P, q);
    BKState& s = S[q];
    const int nv = j + 1, nq = 2 * nv;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    // wave w sums a contiguous quarter of the block partials, lane t output t (each
    // wave reads whole partial rows); the quarters are added in order
    {
        const int per = (p.nblk + NW - 1) / NW;
        const int b0 = wid * per, b1 = min(p.nblk, b0 + per);
        // eight independent partial sums keep eight loads in flight per lane
        double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (lane < nq) {
            const double* src = p.partial + lane;
            int b = b0;
            for (; b + 8 <= b1; b += 8)
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] += src[static_cast<long long>(b + u) * kBKRed];
            for (; b < b1; ++b) a[0] += src[static_cast<long long>(b) * kBKRed];
            part[wid][lane] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
    }
    for (int e = threadIdx.x; e < j * kMB; e += kThreads) {
        const int i = e / kMB, k = e % kMB;
        if (k < i) Ls[e] = s.Lg[i * m + k];
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) a += part[w][threadIdx.x];
        red[threadIdx.x] = a;
    }
    __syncthreads();
    if (wid != 0) return;
    const double sc = lane < nv ? s.scale[lane] : 0.0;
    const double scj = s.scale[j];
    // row j of L
    double l = 0.0;
    if (lane < j) {
        l = sc * scj * red[nv + 1 + lane];
        s.Lg[j * m + lane] = l;
        Ls[j * kMB + lane] = l;
    }
    double amax = fabs(l);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, kWave));
    if (lane == 0) s.orth = fmax(s.orth, amax);
    __builtin_amdgcn_wave_barrier();
    // forward substitution, lane i holding h_i
    double h = 0.0;
    for (int i = 0; i <= j; ++i) {
        const double c = lane < i ? Ls[i * kMB + lane] * h : 0.0;
        const double sum = wave_sum_all(c);
        if (lane == i) h = sc * red[i] - sum;
    }
    if (lane <= j) {
        s.H[lane * m + j] = h;
        s.coef[lane] = sc * h;
    }
}

// w = V_nv -= sum_{i < nv} coef_i V_i;  partial[0] = this block's part of ||w||^2
template <int NVB>
__global__ __launch_bounds__(kThreads) void bk_axpy_norm_kernel(const BKProb* __restrict__ P, const BKState* S,
                                                                int nprob, const int* __restrict__ live, int nv) {
    const LiveBlocks W = prob_live_blocks(P, nprob, live);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const BKProb& p = list_args<BKProb>(P, q);
        double* w = const_cast<double*>(p.v0) + static_cast<long long>(nv) * p.vstride;
        axpy_norm_strided_body<NVB>(p.v0, p.vstride, nv, list_args<BKState>(S, q).coef, w, p.len,
                                    p.partial + static_cast<long long>(local) * kBKRed, local, nb);
        __syncthreads();
    }
}

// Givens update of step j and the convergence test, one workgroup per live problem: a
// problem that reaches the tolerance, the iteration limit or a breakdown leaves the
// cycle (live = 0); otherwise the next basis vector's scale goes to scale[j + 1] and to
// dscale (the input scale of the next forward transform).
__global__ __launch_bounds__(kThreads) void bk_givens_kernel(const BKProb* __restrict__ P, BKState* S, int* live,
                                                             double* dscale, int j, int m, double tol,
                                                             int max_outer) {
    const int q = blockIdx.x;
    if (!live[q]) return;
    __shared__ double col[kMaxBasis], c_s[kMB], s_n[kMB];
    const BKProb& p = list_args<BKProb>(P, q);
    BKState& s = S[q];
    const double hn = sqrt(block_sum_strided(p.partial, p.nblk, kBKRed));
    for (int i = threadIdx.x; i <= j; i += kThreads) {
        col[i] = s.H[i * m + j];
        if (i < j) {
            c_s[i] = s.cs[i];
            s_n[i] = s.sn[i];
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    s.matvecs += s.ell + s.psum;
    if (!isfinite(hn)) {
        s.status = -6;  // AC_ERR_NONFINITE
        s.finished = 1;
        live[q] = 0;
        return;
    }
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = c_s[i] * col[i] + s_n[i] * col[i + 1];
        col[i + 1] = -s_n[i] * col[i] + c_s[i] * col[i + 1];
        col[i] = t;
    }
    const double den = hypot(col[j], col[j + 1]);
    const double cj = den > 0 ? col[j] / den : 1.0;
    const double sj = den > 0 ? col[j + 1] / den : 0.0;
    s.cs[j] = cj;
    s.sn[j] = sj;
    for (int i = 0; i < j; ++i) s.H[i * m + j] = col[i];
    s.H[j * m + j] = den;
    s.H[(j + 1) * m + j] = 0.0;
    const double gj = s.g[j];
    s.g[j + 1] = -sj * gj;
    s.g[j] = cj * gj;
    ++s.total;
    s.kdone = j + 1;
    if (fabs(s.g[j + 1]) / s.bnorm <= tol || s.total >= max_outer || hn == 0.0) {
        live[q] = 0;  // out of this cycle
    } else {
        s.scale[j + 1] = 1.0 / hn;
        dscale[q] = s.scale[j + 1];
    }
}

// End of a cycle, one workgroup per problem in it: y from the triangular system
// H y = g (back substitution).
__global__ __launch_bounds__(kThreads) void bk_backsolve_kernel(BKState* S, const int* __restrict__ cyc, int m) {
    const int q = blockIdx.x;
    if (!cyc[q]) return;
    __shared__ double Hs[kMB * kMB], gs[kMB], ys[kMB];
    BKState& s = S[q];
    const int kd = s.kdone;
    for (int e = threadIdx.x; e < kd * kMB; e += kThreads) {
        const int i = e / kMB, k = e % kMB;
        if (k >= i && k < kd) Hs[e] = s.H[i * m + k];
    }
    for (int i = threadIdx.x; i < kd; i += kThreads) gs[i] = s.g[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = kd - 1; i >= 0; --i) {
        double t = gs[i];
        for (int k = i + 1; k < kd; ++k) t -= Hs[i * kMB + k] * ys[k];
        ys[i] = Hs[i * kMB + i] != 0.0 ? t / Hs[i * kMB + i] : 0.0;
    }
    for (int i = 0; i < kd; ++i) s.y[i] = ys[i];
    ++s.restarts;
}

// x += sum_{i < kdone} y_i Z_i
template <int NVB>
__global__ __launch_bounds__(kThreads) void bk_maxpy_kernel(const BKProb* __restrict__ P, const BKState* S,
                                                            int nprob, const int* __restrict__ cyc) {
    const LiveBlocks W = prob_live_blocks(P, nprob, cyc);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const BKProb& p = list_args<BKProb>(P, q);
        const BKState& st = list_args<BKState>(S, q);
        maxpy_strided_body<NVB>(p.z0, p.vstride, st.kdone, st.y, p.x, p.len, local, nb);
    }
}

// Start of a cycle, one workgroup per problem: for the problems that ran the last
// cycle, ||b - calA x|| from the residual form's tile partials; then the restart test
// and the cycle's initial scalars.  live and cyc mark the problems in the new cycle.
__global__ __launch_bounds__(kThreads) void bk_cycle_kernel(const BKProb* __restrict__ P, BKState* S, int* live,
                                                            int* cyc, double* dscale, int m, double tol,
                                                            int max_outer) {
    const int q = blockIdx.x;
    BKState& s = S[q];
    const bool ran = cyc[q] != 0;
    double rr = 0.0;
    if (ran) rr = block_sum_strided(P[q].partial2, P[q].ntiles, 1);
    __shared__ int go;
    if (threadIdx.x == 0) {
        go = 0;
        if (ran) {
            s.matvecs += s.ell;
            s.beta = sqrt(rr);
        }
        live[q] = 0;
        cyc[q] = 0;
        if (!s.finished) {
            if (!isfinite(s.beta)) {
                s.status = -6;  // AC_ERR_NONFINITE
                s.finished = 1;
            } else if (s.beta / s.bnorm <= tol) {
                s.finished = 1;
            } else if (s.total >= max_outer) {
                s.finished = 1;
                s.status = 1;  // AC_NOT_CONVERGED
            } else {
                go = 1;
            }
        }
    }
    __syncthreads();
    if (!go) return;
    for (int i = threadIdx.x; i < (m + 1) * m; i += kThreads) s.H[i] = 0.0;
    for (int i = threadIdx.x; i <= m; i += kThreads) s.g[i] = i == 0 ? s.beta : 0.0;
    if (threadIdx.x == 0) {
        s.scale[0] = 1.0 / s.beta;
        s.kdone = 0;
        dscale[q] = s.scale[0];
        live[q] = 1;
        cyc[q] = 1;
    }
}

int bucket_nvb(int nv) { return nv <= 4 ? 4 : nv <= 8 ? 8 : nv <= 16 ? 16 : 32; }

}  // namespace

hipError_t launch_bk_mdot(const BKProb* P, int nprob, int blocks, const int* live, int nv, hipStream_t s) {
    if (nv < 1 || nv > kMB || nprob > kListMax) return hipErrorInvalidValue;
    const dim3 g(list_grid(blocks, nprob, kThreads / kWave)), b(kThreads);
    if (nv <= 4) hipLaunchKernelGGL(bk_mdot_kernel<0>, g, b, 0, s, P, nprob, live, nv);
    else if (nv <= 8) hipLaunchKernelGGL(bk_mdot_kernel<1>, g, b, 0, s, P, nprob, live, nv);
    else if (nv <= 16) hipLaunchKernelGGL(bk_mdot_kernel<2>, g, b, 0, s, P, nprob, live, nv);
    else hipLaunchKernelGGL(bk_mdot_kernel<3>, g, b, 0, s, P, nprob, live, nv);
    return hipGetLastError();
}

hipError_t launch_bk_arnoldi(const BKProb* P, BKState* S, int nprob, const int* live, int j, int m, hipStream_t s) {
    if (j < 0 || j >= m || m > kMB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bk_arnoldi_kernel, dim3(nprob), dim3(kThreads), 0, s, P, S, live, j, m);
    return hipGetLastError();
}

hipError_t launch_bk_axpy_norm(const BKProb* P, const BKState* S, int nprob, int blocks, const int* live, int nv,
                               hipStream_t s) {
    if (nv < 1 || nv > kMB || nprob > kListMax) return hipErrorInvalidValue;
    const dim3 g(list_grid(blocks, nprob, kThreads / kWave)), b(kThreads);
    switch (bucket_nvb(nv)) {
        case 4: hipLaunchKernelGGL(bk_axpy_norm_kernel<4>, g, b, 0, s, P, S, nprob, live, nv); break;
        case 8: hipLaunchKernelGGL(bk_axpy_norm_kernel<8>, g, b, 0, s, P, S, nprob, live, nv); break;
        case 16: hipLaunchKernelGGL(bk_axpy_norm_kernel<16>, g, b, 0, s, P, S, nprob, live, nv); break;
        default: hipLaunchKernelGGL(bk_axpy_norm_kernel<32>, g, b, 0, s, P, S, nprob, live, nv); break;
    }
    return hipGetLastError();
}

hipError_t launch_bk_givens(const BKProb* P, BKState* S, int nprob, int* live, double* dscale, int j, int m,
                            double tol, int max_outer, hipStream_t s) {
    if (j < 0 || j >= m || m > kMB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bk_givens_kernel, dim3(nprob), dim3(kThreads), 0, s, P, S, live, dscale, j, m, tol, max_outer);
    return hipGetLastError();
}

hipError_t launch_bk_update(const BKProb* P, BKState* S, int nprob, int blocks, const int* cyc, int m, hipStream_t s) {
    if (m < 1 || m > kMB || nprob > kListMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bk_backsolve_kernel, dim3(nprob), dim3(kThreads), 0, s, S, cyc, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g(list_grid(blocks, nprob, kThreads / kWave)), b(kThreads);
    switch (bucket_nvb(m)) {
        case 4: hipLaunchKernelGGL(bk_maxpy_kernel<4>, g, b, 0, s, P, S, nprob, cyc); break;
        case 8: hipLaunchKernelGGL(bk_maxpy_kernel<8>, g, b, 0, s, P, S, nprob, cyc); break;
        case 16: hipLaunchKernelGGL(bk_maxpy_kernel<16>, g, b, 0, s, P, S, nprob, cyc); break;
        default: hipLaunchKernelGGL(bk_maxpy_kernel<32>, g, b, 0, s, P, S, nprob, cyc); break;
    }
    return hipGetLastError();
}

hipError_t launch_bk_cycle(const BKProb* P, BKState* S, int nprob, int* live, int* cyc, double* dscale, int m,
                           double tol, int max_outer, hipStream_t s) {
    if (m < 1 || m > kMB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bk_cycle_kernel, dim3(nprob), dim3(kThreads), 0, s, P, S, live, cyc, dscale, m, tol,
                       max_outer);
    return hipGetLastError();
}

}  // namespace ac
