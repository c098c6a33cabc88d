// Streaming-bandwidth calibration for the roofline figures: one kernel that reads R and
// writes W contiguous float32x4 streams (R, W in 0..4) in a grid-stride loop, plain loads
// and non-temporal stores, timed with HIP events on the context's stream.  It moves
// exactly the bytes it is given and does no other work, so its rate is the ceiling a
// memory-bound kernel with the same read / write mix can expect on this GPU.
#include <hip/hip_runtime.h>

#include <string>

#include "alphacirc.h"
#include "ac_internal.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int R, int W>
__global__ __launch_bounds__(256) void stream_kernel(f4* base, long long n) {
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < R; ++r) acc += base[static_cast<long long>(r) * n + i];
#pragma unroll
        for (int w = 0; w < W; ++w) __builtin_nontemporal_store(acc + static_cast<float>(w), base + (R + w) * n + i);
        if (W == 0 && acc.x == 1.2345e-30f) base[i] = acc;  // keeps the reads (never taken for zeroed data)
    }
}

template <int R>
hipError_t launch_r(int w, f4* base, long long n, int blocks, hipStream_t s) {
    switch (w) {
        case 0: hipLaunchKernelGGL((stream_kernel<R, 0>), dim3(blocks), dim3(256), 0, s, base, n); break;
        case 1: hipLaunchKernelGGL((stream_kernel<R, 1>), dim3(blocks), dim3(256), 0, s, base, n); break;
        case 2: hipLaunchKernelGGL((stream_kernel<R, 2>), dim3(blocks), dim3(256), 0, s, base, n); break;
        case 3: hipLaunchKernelGGL((stream_kernel<R, 3>), dim3(blocks), dim3(256), 0, s, base, n); break;
        case 4: hipLaunchKernelGGL((stream_kernel<R, 4>), dim3(blocks), dim3(256), 0, s, base, n); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stream(int r, int w, f4* base, long long n, int blocks, hipStream_t s) {
    switch (r) {
        case 0: return launch_r<0>(w, base, n, blocks, s);
        case 1: return launch_r<1>(w, base, n, blocks, s);
        case 2: return launch_r<2>(w, base, n, blocks, s);
        case 3: return launch_r<3>(w, base, n, blocks, s);
        case 4: return launch_r<4>(w, base, n, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int ac_stream_bandwidth(ac_ctx* ctx, int reads, int writes, void* ws, size_t ws_bytes, int reps, double* gbps) {
    if (!ctx || !ws || !gbps) return ac::set_error(AC_ERR_ARG, "NULL argument");
    if (reads < 0 || reads > 4 || writes < 0 || writes > 4 || reads + writes < 1)
        return ac::set_error(AC_ERR_ARG, "reads and writes must be in 0..4, not both zero");
    if (reps < 1) return ac::set_error(AC_ERR_ARG, "reps must be positive");
    const long long n = static_cast<long long>(ws_bytes / 16 / (reads + writes));
    if (n < 1024) return ac::set_error(AC_ERR_WORKSPACE, "workspace too small for the streams");
    if (reinterpret_cast<size_t>(ws) % 16 != 0) return ac::set_error(AC_ERR_ARG, "workspace must be 16-byte aligned");
    const hipStream_t s = ac::ctx_stream(ctx);
    hipError_t e = hipSetDevice(ac::ctx_device(ctx));
    f4* base = static_cast<f4*>(ws);
    const int blocks = 1024;  // four workgroups of 256 threads per CU
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = hipMemsetAsync(ws, 0, static_cast<size_t>(n) * 16 * (reads + writes), s);
    if (e == hipSuccess) e = launch_stream(reads, writes, base, n, blocks, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(t0, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_stream(reads, writes, base, n, blocks, s);
    if (e == hipSuccess) e = hipEventRecord(t1, s);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) return ac::set_error(AC_ERR_HIP, std::string("stream probe: ") + hipGetErrorString(e));
    *gbps = static_cast<double>(n) * 16.0 * (reads + writes) * reps / (ms * 1e-3) / 1e9;
    return AC_OK;
}
