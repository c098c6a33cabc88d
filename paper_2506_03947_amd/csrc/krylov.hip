// Float64 Krylov vector kernels for the outer FGMRES: fused multi-dot,
// multi-axpy with dot or norm, and a deterministic two-stage reduction.
//
// Classical Gram-Schmidt applied twice costs three passes over the basis:
//   (1) d1 = V^T w,  (2) w -= V (s2 .* d1) and d2 = V^T w,  (3) w -= V (s2 .* d2) and ||w||^2,
// where the basis vectors are stored unnormalised and s2_i is the square of their
// scale (so no pass is spent normalising).  Each thread keeps the basis values of
// its two elements in registers between the axpy and the following dot.
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr int kBlocks = 1024;
constexpr int kThreads = 256;

struct alignas(16) D2 {
    double x, y;
};

__device__ __forceinline__ D2 load2(const double* p, long long e, long long len) {
    D2 r;
    if (e + 1 < len) {
        r = *reinterpret_cast<const D2*>(p + e);
    } else {
        r.x = p[e];
        r.y = 0.0;
    }
    return r;
}
__device__ __forceinline__ void store2(double* p, long long e, long long len, D2 v) {
    if (e + 1 < len) {
        *reinterpret_cast<D2*>(p + e) = v;
    } else {
        p[e] = v.x;
    }
}

// Block-wide sums of NQ per-thread values; thread q < nq writes partial[q].
template <int NQ>
__device__ __forceinline__ void block_sums(double (&acc)[NQ], int nq, double* partial) {
    __shared__ double red[kThreads / kWave][NQ];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
        if (lane == 0) red[wid][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / kWave; ++w) s += red[w][threadIdx.x];
        partial[threadIdx.x] = s;
    }
}

template <int NVB>
__global__ __launch_bounds__(kThreads) void mdot_kernel(const VecSet V, int nv, const double* __restrict__ w,
                                                        long long len, double* partial, int stride) {
    double acc[NVB];
#pragma unroll
    for (int i = 0; i < NVB; ++i) acc[i] = 0.0;
    const long long step = 2LL * gridDim.x * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x); e < len; e += step) {
        const D2 wv = load2(w, e, len);
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            if (i < nv) {
                const D2 v = load2(V.v[i], e, len);
                acc[i] += v.x * wv.x + v.y * wv.y;
            }
        }
    }
    block_sums<NVB>(acc, nv, partial + static_cast<long long>(blockIdx.x) * stride);
}

template <int NVB, bool DOT>
__global__ __launch_bounds__(kThreads) void axpy_kernel(const VecSet V, int nv, const double* __restrict__ dcoef,
                                                        double* w, long long len, double* partial, int stride) {
    double coef[NVB];
#pragma unroll
    for (int i = 0; i < NVB; ++i) coef[i] = (i < nv) ? V.s2[i] * dcoef[i] : 0.0;
    constexpr int NQ = DOT ? NVB : 1;
    double acc[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
    const long long step = 2LL * gridDim.x * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x); e < len; e += step) {
        D2 wv = load2(w, e, len);
        D2 vv[NVB];
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            if (i < nv) {
                vv[i] = load2(V.v[i], e, len);
                wv.x -= coef[i] * vv[i].x;
                wv.y -= coef[i] * vv[i].y;
            }
        }
        store2(w, e, len, wv);
        if (DOT) {
#pragma unroll
            for (int i = 0; i < NVB; ++i)
                if (i < nv) acc[i < NQ ? i : 0] += vv[i].x * wv.x + vv[i].y * wv.y;
        } else {
            acc[0] += wv.x * wv.x + wv.y * wv.y;
        }
    }
    block_sums<NQ>(acc, DOT ? nv : 1, partial + static_cast<long long>(blockIdx.x) * stride);
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

hipError_t launch_mdot(const VecSet& V, int nv, const double* w, long long len, double* partial, int stride,
                       hipStream_t s) {
    if (nv < 1 || nv > 32) return hipErrorInvalidValue;
    switch (bucket(nv)) {
        case 4: hipLaunchKernelGGL(mdot_kernel<4>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, w, len, partial, stride); break;
        case 8: hipLaunchKernelGGL(mdot_kernel<8>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, w, len, partial, stride); break;
        case 16: hipLaunchKernelGGL(mdot_kernel<16>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, w, len, partial, stride); break;
        default: hipLaunchKernelGGL(mdot_kernel<32>, dim3(kBlocks), dim3(kThreads), 0, s, V, nv, w, len, partial, stride); break;
    }
    return hipGetLastError();
}

hipError_t launch_axpy_dot(const VecSet& V, int nv, const double* dcoef, double* w, long long len, double* partial,
                           int stride, hipStream_t s) {
    if (nv < 1 || nv > 32) return hipErrorInvalidValue;
    switch (bucket(nv)) {
        case 4: hipLaunchKernelGGL((axpy_kernel<4, true>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        case 8: hipLaunchKernelGGL((axpy_kernel<8, true>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        case 16: hipLaunchKernelGGL((axpy_kernel<16, true>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        default: hipLaunchKernelGGL((axpy_kernel<32, true>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
    }
    return hipGetLastError();
}

hipError_t launch_axpy_norm(const VecSet& V, int nv, const double* dcoef, double* w, long long len, double* partial,
                            int stride, hipStream_t s) {
    if (nv < 1 || nv > 32) return hipErrorInvalidValue;
    switch (bucket(nv)) {
        case 4: hipLaunchKernelGGL((axpy_kernel<4, false>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        case 8: hipLaunchKernelGGL((axpy_kernel<8, false>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        case 16: hipLaunchKernelGGL((axpy_kernel<16, false>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
        default: hipLaunchKernelGGL((axpy_kernel<32, false>), dim3(kBlocks), dim3(kThreads), 0, s, V, nv, dcoef, w, len, partial, stride); break;
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

hipError_t launch_norm2(const double* w, long long len, double* partial, hipStream_t s) {
    hipLaunchKernelGGL(norm2_kernel, dim3(kBlocks), dim3(kThreads), 0, s, w, len, partial);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int nblk, int nq, int stride, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(nq), dim3(kThreads), 0, s, partial, nblk, stride, out);
    return hipGetLastError();
}

}  // namespace ac
