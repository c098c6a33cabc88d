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

namespace ac {
namespace {

constexpr int kBlocks = 1024;
constexpr int kThreads = 256;

struct alignas(16) D2 {
    double x, y;
};

// Krylov vectors are far larger than the caches between two uses: stream them.
typedef double D2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ D2 load2(const double* p, long long e, long long len) {
    D2 r;
    if (e + 1 < len) {
        const D2v t = __builtin_nontemporal_load(reinterpret_cast<const D2v*>(p + e));
        r.x = t[0];
        r.y = t[1];
    } else {
        r.x = p[e];
        r.y = 0.0;
    }
    return r;
}
// Same, zero past the end (the second element of an unrolled pair of iterations).
__device__ __forceinline__ D2 load2z(const double* p, long long e, long long len) {
    if (e < len) return load2(p, e, len);
    return D2{0.0, 0.0};
}
// Cached load for an operand that every wave of a block reads (the multi-dot's target
// and newest basis vector): the block's other waves then hit L2 instead of HBM.
__device__ __forceinline__ D2 load2c(const double* p, long long e, long long len) {
    if (e + 1 < len) {
        const D2v t = *reinterpret_cast<const D2v*>(p + e);
        return D2{t[0], t[1]};
    }
    if (e < len) return D2{p[e], 0.0};
    return D2{0.0, 0.0};
}
__device__ __forceinline__ void store2(double* p, long long e, long long len, D2 v) {
    if (e + 1 < len) {
        D2v t;
        t[0] = v.x;
        t[1] = v.y;
        __builtin_nontemporal_store(t, reinterpret_cast<D2v*>(p + e));
    } else {
        p[e] = v.x;
    }
}

// Block-wide sums of NQ per-thread values; thread q < nq writes partial[q] from
// accumulator src(q) = q, except that q == remap_from reads accumulator NQ-1.
template <int NQ>
__device__ __forceinline__ void block_sums(double (&acc)[NQ], int nq, double* partial, int remap_from = -1) {
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
        const int src = (static_cast<int>(threadIdx.x) == remap_from) ? NQ - 1 : threadIdx.x;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / kWave; ++w) s += red[w][src];
        partial[threadIdx.x] = s;
    }
}

// Block sums for mdot: out[q] for q < nv from acc[q], out[nv] from acc[NVB], and
// (TWO) out[nv + 1 + q] for q < nv - 1 from acc[NVB + 1 + q].
template <int NQ, int NVB, bool TWO>
__device__ __forceinline__ void block_sums_mdot(double (&acc)[NQ], int nv, double* partial) {
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
    const int nout = TWO ? 2 * nv : nv + 1;
    const int t = threadIdx.x;
    if (t < nout) {
        const int src = (t < nv) ? t : (t == nv ? NVB : NVB + 1 + (t - nv - 1));
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / kWave; ++w) s += red[w][src];
        partial[t] = s;
    }
}

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

// Vector-parallel multi-dot for a basis stored with a fixed stride (V_i = V_0 + i*vstride):
// the waves of a block walk the same element chunk, wave g owning basis vectors
// [g*G, g*G + G), so each thread keeps at most 2G accumulators; the shared operands
// w (and v_last) are re-read by the four waves from L1/L2, not from HBM.
// Outputs as mdot_kernel: q < nv: V_q . w;  nv: w . w;  (TWO) nv + 1 + q: V_q . V_{nv-1}.
template <int G, bool TWO>
__global__ __launch_bounds__(kThreads) void mdot_vp_kernel(const double* __restrict__ v0, long long vstride, int nv,
                                                           const double* __restrict__ w, long long len,
                                                           double* partial, int stride) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i0 = wid * G;
    double acc[G], acc2[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = acc2[g] = 0.0;
    double nrm = 0.0;
    const double* __restrict__ vl = v0 + static_cast<long long>(nv - 1) * vstride;
    const long long step = 2LL * kWave * gridDim.x;
    // two iterations per trip (G <= 4; more would cost occupancy): all their loads are
    // issued before the first product, and the sums are taken in the plain loop's order
    constexpr int U = G <= 4 ? 2 : 1;
    for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * kWave + lane); e < len; e += U * step) {
        const long long e2 = U == 2 ? e + step : len;
        const D2 wv = load2c(w, e, len);
        const D2 wv2 = load2c(w, e2, len);
        D2 lv{0.0, 0.0}, lv2{0.0, 0.0};
        if (TWO) {
            lv = load2c(vl, e, len);
            lv2 = load2c(vl, e2, len);
        }
        D2 v[G], v2[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            v[g] = v2[g] = D2{0.0, 0.0};
            if (i0 + g < nv) {
                v[g] = load2(v0 + static_cast<long long>(i0 + g) * vstride, e, len);
                v2[g] = load2z(v0 + static_cast<long long>(i0 + g) * vstride, e2, len);
            }
        }
        if (wid == 0) {
            nrm += wv.x * wv.x + wv.y * wv.y;
            nrm += wv2.x * wv2.x + wv2.y * wv2.y;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (i0 + g < nv) {
                acc[g] += v[g].x * wv.x + v[g].y * wv.y;
                if (TWO) acc2[g] += v[g].x * lv.x + v[g].y * lv.y;
                acc[g] += v2[g].x * wv2.x + v2[g].y * wv2.y;
                if (TWO) acc2[g] += v2[g].x * lv2.x + v2[g].y * lv2.y;
            }
        }
    }
    double* out = partial + static_cast<long long>(blockIdx.x) * stride;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double a = acc[g], b = acc2[g];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            a += __shfl_down(a, off, kWave);
            if (TWO) b += __shfl_down(b, off, kWave);
        }
        if (lane == 0 && i0 + g < nv) out[i0 + g] = a;
        if (TWO && lane == 0 && i0 + g < nv - 1) out[nv + 1 + i0 + g] = b;
    }
    if (wid == 0) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) nrm += __shfl_down(nrm, off, kWave);
        if (lane == 0) out[nv] = nrm;
    }
}

// w -= sum_i c_i V_i with c_i = s2_i dcoef_i (dcoef on the device) or c_i = s2_i
// (dcoef == nullptr);  partial[0] = ||w||^2 afterwards
// Few basis vectors (nv <= NVB, 4 or 8, contiguous at a stride): every thread streams its
// own elements of w and of all nv vectors (no wave re-reads w), two iterations per trip;
// the dots with the newest vector come from the same loads.  Partial layout as above.
template <int NVB, bool TWO>
__global__ __launch_bounds__(kThreads) void mdot_es_kernel(const double* __restrict__ v0, long long vstride, int nv,
                                                           const double* __restrict__ w, long long len,
                                                           double* partial, int stride) {
    constexpr int NQ = 2 * NVB + 1;
    double acc[NQ];  // [0, NVB): V_i . w; NVB: w . w; NVB + 1 + i: V_i . V_{nv-1}
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
    const long long step = 2LL * gridDim.x * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x); e < len; e += 2 * step) {
        const long long e2 = e + step;
        const D2 wv = load2(w, e, len);
        const D2 wv2 = load2z(w, e2, len);
        D2 v[NVB], v2[NVB];
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            v[i] = v2[i] = D2{0.0, 0.0};
            if (i < nv) {
                v[i] = load2(v0 + static_cast<long long>(i) * vstride, e, len);
                v2[i] = load2z(v0 + static_cast<long long>(i) * vstride, e2, len);
            }
        }
        D2 lv = v[0], lv2 = v2[0];
#pragma unroll
        for (int i = 1; i < NVB; ++i)
            if (i == nv - 1) {
                lv = v[i];
                lv2 = v2[i];
            }
        acc[NVB] += wv.x * wv.x + wv.y * wv.y;
        acc[NVB] += wv2.x * wv2.x + wv2.y * wv2.y;
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            if (i < nv) {
                acc[i] += v[i].x * wv.x + v[i].y * wv.y;
                if (TWO) acc[NVB + 1 + i] += v[i].x * lv.x + v[i].y * lv.y;
                acc[i] += v2[i].x * wv2.x + v2[i].y * wv2.y;
                if (TWO) acc[NVB + 1 + i] += v2[i].x * lv2.x + v2[i].y * lv2.y;
            }
        }
    }
    block_sums_mdot<NQ, NVB, TWO>(acc, nv, partial + static_cast<long long>(blockIdx.x) * stride);
}

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
