// Float64 Krylov vector bodies shared by the single-problem kernels (krylov.hip) and
// the batched ones (batch_krylov.hip): a body covers the elements of block `bid` of
// `nb` blocks and writes that block's partial sums to `out`, so the same arithmetic
// serves one grid per problem and a work list of problems.  Krylov vectors are far
// larger than the caches between two uses: they are streamed.
#pragma once

#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace kry {

constexpr int kThreads = 256;

struct alignas(16) D2 {
    double x, y;
};

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

// Vector-parallel multi-dot for a basis stored with a fixed stride (V_i = V_0 + i*vstride):
// the waves of a block walk the same element chunk, wave g owning basis vectors
// [g*G, g*G + G), so each thread keeps at most 2G accumulators; the shared operands
// w (and v_last) are re-read by the four waves from L1/L2, not from HBM.
// Outputs as mdot_kernel: q < nv: V_q . w;  nv: w . w;  (TWO) nv + 1 + q: V_q . V_{nv-1}.
template <int G, bool TWO>
__device__ __forceinline__ void mdot_vp_body(const double* __restrict__ v0, long long vstride, int nv,
                                             const double* __restrict__ w, long long len, double* out, int bid,
                                             int nb) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i0 = wid * G;
    double acc[G], acc2[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = acc2[g] = 0.0;
    double nrm = 0.0;
    const double* __restrict__ vl = v0 + static_cast<long long>(nv - 1) * vstride;
    const long long step = 2LL * kWave * nb;
    // two iterations per trip (G <= 4; more would cost occupancy): all their loads are
    // issued before the first product, and the sums are taken in the plain loop's order
    constexpr int U = G <= 4 ? 2 : 1;
    for (long long e = 2LL * (static_cast<long long>(bid) * kWave + lane); e < len; e += U * step) {
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

// Few basis vectors (nv <= NVB, 4 or 8, contiguous at a stride): every thread streams its
// own elements of w and of all nv vectors (no wave re-reads w), two iterations per trip;
// the dots with the newest vector come from the same loads.  Partial layout as above.
template <int NVB, bool TWO>
__device__ __forceinline__ void mdot_es_body(const double* __restrict__ v0, long long vstride, int nv,
                                             const double* __restrict__ w, long long len, double* out, int bid,
                                             int nb) {
    constexpr int NQ = 2 * NVB + 1;
    double acc[NQ];  // [0, NVB): V_i . w; NVB: w . w; NVB + 1 + i: V_i . V_{nv-1}
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
    const long long step = 2LL * nb * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(bid) * blockDim.x + threadIdx.x); e < len; e += 2 * step) {
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
    block_sums_mdot<NQ, NVB, TWO>(acc, nv, out);
}

// Strided basis (V_i = v0 + i * vstride): w -= sum_{i < nv} coef_i V_i, then out[0] =
// this block's part of ||w||^2.
template <int NVB>
__device__ __forceinline__ void axpy_norm_strided_body(const double* __restrict__ v0, long long vstride, int nv,
                                                       const double* __restrict__ dcoef, double* w, long long len,
                                                       double* out, int bid, int nb) {
    double coef[NVB];
#pragma unroll
    for (int i = 0; i < NVB; ++i) coef[i] = (i < nv) ? dcoef[i] : 0.0;
    double acc[1] = {0.0};
    const long long step = 2LL * nb * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(bid) * blockDim.x + threadIdx.x); e < len; e += step) {
        D2 wv = load2(w, e, len);
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            if (i < nv) {
                const D2 v = load2(v0 + static_cast<long long>(i) * vstride, e, len);
                wv.x -= coef[i] * v.x;
                wv.y -= coef[i] * v.y;
            }
        }
        store2(w, e, len, wv);
        acc[0] += wv.x * wv.x + wv.y * wv.y;
    }
    block_sums<1>(acc, 1, out);
}

// Strided vectors Z_i = z0 + i * vstride: x += sum_{i < nv} y_i Z_i
template <int NVB>
__device__ __forceinline__ void maxpy_strided_body(const double* __restrict__ z0, long long vstride, int nv,
                                                   const double* __restrict__ dy, double* x, long long len, int bid,
                                                   int nb) {
    double y[NVB];
#pragma unroll
    for (int i = 0; i < NVB; ++i) y[i] = (i < nv) ? dy[i] : 0.0;
    const long long step = 2LL * nb * blockDim.x;
    for (long long e = 2LL * (static_cast<long long>(bid) * blockDim.x + threadIdx.x); e < len; e += step) {
        D2 xv = load2(x, e, len);
#pragma unroll
        for (int i = 0; i < NVB; ++i) {
            if (i < nv) {
                const D2 v = load2(z0 + static_cast<long long>(i) * vstride, e, len);
                xv.x += y[i] * v.x;
                xv.y += y[i] * v.y;
            }
        }
        store2(x, e, len, xv);
    }
}

}  // namespace kry
}  // namespace ac
