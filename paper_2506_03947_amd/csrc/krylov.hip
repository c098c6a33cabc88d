// Float64 Krylov vector kernels for the outer FGMRES: fused multi-dot (with the
// norm of the target), multi-axpy with the norm of the result, and a
// deterministic two-stage reduction.
//
// One Gram-Schmidt step costs two sweeps over the basis:
//   (1) d = V^T w, ||w||^2 and (optionally) e = V^T v_last, the dots of the newest
//       basis vector with the older ones (free: v_last is read anyway),
//   (2) w -= V c and ||w||^2 with host-computed coefficients c,
// where the basis vectors are stored unnormalised (the host keeps their scales,
// so no sweep is spent normalising).
#include <hip/hip_runtime.h>

#include "ac_internal.h"
#include "krylov_body.h"

namespace ac {
namespace {

using namespace kry;

constexpr int kBlocks = 1024;

// partial[q], q < nv: V_q . w;  partial[nv]: w . w;
// TWO: partial[nv + 1 + q], q < nv - 1: V_q . V_{nv-1}
template <int NVB, bool TWO>
__global__ __launch_bounds__(kThreads) void mdot_kernel(const VecSet V, int nv, const double* __restrict__ w,
                                                        long long len, double* partial, int stride) {
    constexpr int NQ = TWO ? 2 * NVB + 1 : NVB + 1;
    double acc[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
    if (TWO) {
        // one element per thread per step keeps the two accumulator sets in registers
        const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
        const double* __restrict__ vl = V.v[nv - 1];
        for (long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; e < len; e += step) {
            const double wv = w[e];
            const double lv = vl[e];
            acc[NVB] += wv * wv;
#pragma unroll
            for (int i = 0; i < NVB; ++i) {
                if (i < nv) {
                    const double v = V.v[i][e];
                    acc[i] += v * wv;
                    if (TWO && i < NVB) acc[(NVB + 1 + i) % NQ] += v * lv;
                }
            }
        }
    } else {
        const long long step = 2LL * gridDim.x * blockDim.x;
        for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x); e < len;
             e += step) {
            const D2 wv = load2(w, e, len);
            acc[NVB] += wv.x * wv.x + wv.y * wv.y;
#pragma unroll
            for (int i = 0; i < NVB; ++i) {
                if (i < nv) {
                    const D2 v = load2(V.v[i], e, len);
                    acc[i] += v.x * wv.x + v.y * wv.y;
                }
            }
        }
    }
    block_sums_mdot<NQ, NVB, TWO>(acc, nv, partial + static_cast<long long>(blockIdx.x) * stride);
}

// Vector-parallel multi-dot over a strided basis (mdot_vp_body)
template <int G, bool TWO>
__global__ __launch_bounds__(kThreads) void mdot_vp_kernel(const double* __restrict__ v0, long long vstride, int nv,
                                                           const double* __restrict__ w, long long len,
                                                           double* partial, int stride) {
    mdot_vp_body<G, TWO>(v0, vstride, nv, w, len, partial + static_cast<long long>(blockIdx.x) * stride, blockIdx.x,
                         gridDim.x);
}

// Few basis vectors, element-split over the threads (mdot_es_body)
template <int NVB, bool TWO>
__global__ __launch_bounds__(kThreads) void mdot_es_kernel(const double* __restrict__ v0, long long vstride, int nv,
                                                           const double* __restrict__ w, long long len,
                                                           double* partial, int stride) {
    mdot_es_body<NVB, TWO>(v0, vstride, nv, w, len, partial + static_cast<long long>(blockIdx.x) * stride, blockIdx.x,
                           gridDim.x);
}

// w -= sum_i c_i V_i with c_i = s2_i dcoef_i (dcoef on the device) or c_i = s2_i
// (dcoef == nullptr);  partial[0] = ||w||^2 afterwards
template <int NVB>
__global__ __launch_bounds__(kThreads) void axpy_norm_kernel(const VecSet V, int nv, const double* __restrict__ dcoef,
                                                             double* w, long long len, double* partial, int stride) {
    double coef[NVB];
#pragma unroll
    for (int i = 0; i < NVB; ++i) coef[i] = (i < nv) ? (dcoef ? V.s2[i] * dcoef[i] : V.s2[i]) : 0.0;
    double acc[1] = {0.0};
    const long long step = 2LL * gridDim.x * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x); e < len; e += step) {
        D2 wv = load2(w, e, len);
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            if (i < nv) {
                const D2 v = load2(V.v[i], e, len);
                wv.x -= coef[i] * v.x;
                wv.y -= coef[i] * v.y;
            }
        }
        store2(w, e, len, wv);
        acc[0] += wv.x * wv.x + wv.y * wv.y;
    }
    block_sums<1>(acc, 1, partial + static_cast<long long>(blockIdx.x) * stride);
}

template <int NVB>
__global__ __launch_bounds__(kThreads) void maxpy_kernel(const VecSet Z, int nv, double* x, long long len) {
    const long long step = 2LL * gridDim.x * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x); e < len; e += step) {
        D2 xv = load2(x, e, len);
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            if (i < nv) {
                const D2 v = load2(Z.v[i], e, len);
                xv.x += Z.s2[i] * v.x;
                xv.y += Z.s2[i] * v.y;
            }
        }
        store2(x, e, len, xv);
    }
}

__global__ __launch_bounds__(kThreads) void norm2_kernel(const double* __restrict__ w, long long len,
                                                         double* partial) {
    double acc[1] = {0.0};
    const long long step = 2LL * gridDim.x * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x); e < len; e += step) {
        const D2 v = load2(w, e, len);
        acc[0] += v.x * v.x + v.y * v.y;
    }
    block_sums<1>(acc, 1, partial + blockIdx.x);
}

// out[q] = sum_b partial[b*stride + q], one block per q, fixed order.
__global__ __launch_bounds__(kThreads) void reduce_kernel(const double* __restrict__ partial, int nblk, int stride,
                                                          double* out) {
    const int q = blockIdx.x;
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc[0] += partial[static_cast<long long>(b) * stride + q];
    block_sums<1>(acc, 1, out + q);
}

int bucket(int nv) { return nv <= 4 ? 4 : nv <= 8 ? 8 : nv <= 16 ? 16 : 32; }

}  // namespace

int krylov_blocks() { return kBlocks; }

hipError_t launch_mdot(const VecSet& V, int nv, bool with_last, const double* w, long long len, double* partial,
                       int stride, hipStream_t s) {
    if (nv < 1 || nv > 32) return hipErrorInvalidValue;
    const dim3 g(kBlocks), b(kThreads);
#define AC_MD(NB)                                                                                   \
    if (with_last) hipLaunchKernelGGL((mdot_kernel<NB, true>), g, b, 0, s, V, nv, w, len, partial, stride); \
    else hipLaunchKernelGGL((mdot_kernel<NB, false>), g, b, 0, s, V, nv, w, len, partial, stride);
    switch (bucket(nv)) {
        case 4: AC_MD(4) break;
        case 8: AC_MD(8) break;
        case 16: AC_MD(16) break;
        default: AC_MD(32) break;
    }
#undef AC_MD
    return hipGetLastError();
}

hipError_t launch_mdot_strided(const double* v0, long long vstride, int nv, bool with_last, const double* w,
                               long long len, double* partial, int stride, hipStream_t s) {
    if (nv < 1 || nv > 32) return hipErrorInvalidValue;
    const int per_wave = (nv + kThreads / kWave - 1) / (kThreads / kWave);
    const dim3 g(kBlocks), b(kThreads);
    if (nv <= 4) {  // few vectors: split the elements, not the vectors, over the waves
        if (with_last) hipLaunchKernelGGL((mdot_es_kernel<4, true>), g, b, 0, s, v0, vstride, nv, w, len, partial, stride);
        else hipLaunchKernelGGL((mdot_es_kernel<4, false>), g, b, 0, s, v0, vstride, nv, w, len, partial, stride);
        return hipGetLastError();
    }
    if (nv <= 8) {
        if (with_last) hipLaunchKernelGGL((mdot_es_kernel<8, true>), g, b, 0, s, v0, vstride, nv, w, len, partial, stride);
        else hipLaunchKernelGGL((mdot_es_kernel<8, false>), g, b, 0, s, v0, vstride, nv, w, len, partial, stride);
        return hipGetLastError();
    }
#define AC_MV(GG)                                                                                             \
    if (with_last) hipLaunchKernelGGL((mdot_vp_kernel<GG, true>), g, b, 0, s, v0, vstride, nv, w, len, partial, stride); \
    else hipLaunchKernelGGL((mdot_vp_kernel<GG, false>), g, b, 0, s, v0, vstride, nv, w, len, partial, stride);
    if (per_wave <= 1) { AC_MV(1) }
    else if (per_wave <= 2) { AC_MV(2) }
    else if (per_wave <= 4) { AC_MV(4) }
    else { AC_MV(8) }
#undef AC_MV
    return hipGetLastError();
}

hipError_t launch_axpy_norm(const VecSet& V, int nv, const double* dcoef, double* w, long long len, double* partial,
                            int stride, hipStream_t s) {
    if (nv < 1 || nv > 32) return hipErrorInvalidValue;
    switch (bucket(nv)) {
        case 4: hipLaunchKernelGGL(axpy_norm_kernel<4>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        case 8: hipLaunchKernelGGL(axpy_norm_kernel<8>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        case 16: hipLaunchKernelGGL(axpy_norm_kernel<16>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        default: hipLaunchKernelGGL(axpy_norm_kernel<32>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
    }
    return hipGetLastError();
}

hipError_t launch_maxpy(const VecSet& Z, int nv, const double* /*unused*/, double* x, long long len, hipStream_t s) {
    if (nv < 1 || nv > 32) return hipErrorInvalidValue;
    switch (bucket(nv)) {
        case 4: hipLaunchKernelGGL(maxpy_kernel<4>, dim3(kBlocks), dim3(kThreads), 0, s, Z, nv, x, len); break;
        case 8: hipLaunchKernelGGL(maxpy_kernel<8>, dim3(kBlocks), dim3(kThreads), 0, s, Z, nv, x, len); break;
        case 16: hipLaunchKernelGGL(maxpy_kernel<16>, dim3(kBlocks), dim3(kThreads), 0, s, Z, nv, x, len); break;
        default: hipLaunchKernelGGL(maxpy_kernel<32>, dim3(kBlocks), dim3(kThreads), 0, s, Z, nv, x, len); break;
    }
    return hipGetLastError();
}

// Outer Chebyshev update: d = a d + c z, then x = x + d.
__global__ __launch_bounds__(256) void cheb_update_kernel(double* __restrict__ x, double* __restrict__ d,
                                                          const double* __restrict__ z, double a, double c,
                                                          long long len) {
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += step) {
        const double dn = c * z[i] + (a != 0.0 ? a * d[i] : 0.0);  // d is not read on the first step
        d[i] = dn;
        x[i] += dn;
    }
}

hipError_t launch_cheb_update(double* x, double* d, const double* z, double a, double c, long long len,
                              hipStream_t s) {
    hipLaunchKernelGGL(cheb_update_kernel, dim3(kBlocks), dim3(kThreads), 0, s, x, d, z, a, c, len);
    return hipGetLastError();
}

hipError_t launch_norm2(const double* w, long long len, double* partial, hipStream_t s) {
    hipLaunchKernelGGL(norm2_kernel, dim3(kBlocks), dim3(kThreads), 0, s, w, len, partial);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int nblk, int nq, int stride, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(nq), dim3(kThreads), 0, s, partial, nblk, stride, out);
    return hipGetLastError();
}

}  // namespace ac
