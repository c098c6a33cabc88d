// Problem set-up kernels: coefficient copies for the mixed-precision inner solve
// and the reductions behind the enclosing spectral interval.
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr int kBlocks = 512;
constexpr int kThreads = 256;
constexpr int kNQ = 8;

// float -> bfloat16 bits, round to nearest even (inputs are finite here)
__device__ __forceinline__ uint16_t to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ double from_bf16(uint16_t b) {
    return static_cast<double>(__uint_as_float(static_cast<uint32_t>(b) << 16));
}

// Gershgorin value of row i (centre + radius) for a kappa accessor.
template <typename F>
__device__ double gersh(const Geom& g, int ix, int iy, F kap) {
    const double kc = kap(ix, iy);
    double all = 0.0, interior = 0.0;
    const int ndir = g.dim == 2 ? 4 : 2;
    const int dx[4] = {1, -1, 0, 0};
    const int dy[4] = {0, 0, 1, -1};
    for (int d = 0; d < ndir; ++d) {
        int jx = ix + dx[d], jy = iy + dy[d];
        const bool inside = jx >= 0 && jx < g.nx && jy >= 0 && jy < g.ny;
        if (inside || g.periodic) {
            jx = (jx + g.nx) % g.nx;
            jy = (jy + g.ny) % g.ny;
            const double kf = 0.5 * (kc + kap(jx, jy));
            all += kf;
            // a periodic face onto the cell itself (n = 1 along that axis) cancels
            if (!(jx == ix && jy == iy)) interior += kf;
            else all -= kf;
        } else {
            all += kc;
        }
    }
    return 1.0 + all + interior;
}

__global__ __launch_bounds__(kThreads) void kappa_setup_kernel(const Geom g, const double* __restrict__ k64,
                                                               float* k32, uint16_t* k16, double* partial) {
    // q: 0 min k64, 1 max gersh64, 2 min k32, 3 max gersh32, 4 min k16, 5 max gersh16, 6 bad count, 7 max k64
    double acc[kNQ] = {1e308, 0.0, 1e308, 0.0, 1e308, 0.0, 0.0, 0.0};
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < g.n; i += step) {
        const double k = k64[i];
        const bool ok = (k > 0.0) && (k < 1e300);
        acc[6] += ok ? 0.0 : 1.0;
        const float kf = static_cast<float>(k);
        k32[i] = kf;
        const uint16_t kb = to_bf16_rne(kf);
        k16[i] = kb;
        const int ix = static_cast<int>(i % g.nx), iy = static_cast<int>(i / g.nx);
        auto a64 = [&](int x, int y) { return k64[static_cast<long long>(y) * g.nx + x]; };
        auto a32 = [&](int x, int y) { return static_cast<double>(static_cast<float>(k64[static_cast<long long>(y) * g.nx + x])); };
        auto a16 = [&](int x, int y) {
            return from_bf16(to_bf16_rne(static_cast<float>(k64[static_cast<long long>(y) * g.nx + x])));
        };
        acc[0] = fmin(acc[0], k);
        acc[7] = fmax(acc[7], k);
        acc[1] = fmax(acc[1], gersh(g, ix, iy, a64));
        acc[2] = fmin(acc[2], static_cast<double>(kf));
        acc[3] = fmax(acc[3], gersh(g, ix, iy, a32));
        acc[4] = fmin(acc[4], from_bf16(kb));
        acc[5] = fmax(acc[5], gersh(g, ix, iy, a16));
    }
    __shared__ double red[kThreads / kWave][kNQ];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    for (int q = 0; q < kNQ; ++q) {
        double v = acc[q];
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double o = __shfl_down(v, off, kWave);
            v = (q == 6) ? v + o : (q % 2 == 0 ? fmin(v, o) : fmax(v, o));
        }
        if (lane == 0) red[wid][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNQ) {
        const int q = threadIdx.x;
        double v = red[0][q];
        for (int w = 1; w < kThreads / kWave; ++w)
            v = (q == 6) ? v + red[w][q] : (q % 2 == 0 ? fmin(v, red[w][q]) : fmax(v, red[w][q]));
        partial[blockIdx.x * kNQ + q] = v;
    }
}

// Pointwise mean of l coefficient fields (block-major) and per-block counts of
// entries that are not finite and positive.
__global__ __launch_bounds__(kThreads) void kappa_mean_kernel(const double* __restrict__ kb, int ell, long long n,
                                                              double* __restrict__ mean, double* __restrict__ bad) {
    double nbad = 0.0;
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) {
        double s = 0.0;
        for (int k = 0; k < ell; ++k) {
            const double v = kb[static_cast<long long>(k) * n + i];
            if (!(v > 0.0 && v < 1.0e300)) nbad += 1.0;
            s += v;
        }
        mean[i] = s / ell;
    }
    __shared__ double red[kThreads / 64];
    for (int off = 32; off > 0; off >>= 1) nbad += __shfl_down(nbad, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nbad;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += red[w];
        bad[blockIdx.x] = t;
    }
}

}  // namespace

int setup_blocks() { return kBlocks; }

hipError_t launch_kappa_setup(const Geom& g, const double* kappa, float* k32, uint16_t* k16, double* partial,
                              int nblk, hipStream_t s) {
    hipLaunchKernelGGL(kappa_setup_kernel, dim3(nblk), dim3(kThreads), 0, s, g, kappa, k32, k16, partial);
    return hipGetLastError();
}

hipError_t launch_kappa_mean(const double* kb, int ell, long long n, double* mean, double* bad, hipStream_t s) {
    hipLaunchKernelGGL(kappa_mean_kernel, dim3(kBlocks), dim3(kThreads), 0, s, kb, ell, n, mean, bad);
    return hipGetLastError();
}

}  // namespace ac
