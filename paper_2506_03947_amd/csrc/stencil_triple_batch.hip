// Batched (work-list) launches of the three-step shifted-Chebyshev sweep over many
// problems of uneven size (the device body is in stencil_triple.h).
#include "stencil_triple.h"

namespace ac {
namespace {

template <typename R, typename KS, int VX, bool FIRST>
hipError_t batch_triple_kind(int kind, const BatchList& L, hipStream_t s) {
    const dim3 grid(L.blocks), block(L.wpb * kWave);
    if (kind == 0) hipLaunchKernelGGL((cheb_triple_batch_kernel<R, KS, VX, 2, 1, FIRST>), grid, block, 0, s, L);
    else hipLaunchKernelGGL((cheb_triple_batch_kernel<R, KS, VX, 1, 2, FIRST>), grid, block, 0, s, L);
    return hipGetLastError();
}

template <typename R, typename KS>
hipError_t batch_triple_t(int code, int vx, const BatchList& L, hipStream_t s) {
    const int kind = code & 1;
    const bool first = (code & 2) != 0;
    if (vx == 2) return first ? batch_triple_kind<R, KS, 2, true>(kind, L, s) : batch_triple_kind<R, KS, 2, false>(kind, L, s);
    if (vx == 1) return first ? batch_triple_kind<R, KS, 1, true>(kind, L, s) : batch_triple_kind<R, KS, 1, false>(kind, L, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batch_triple(int prec, int code, int vx, const BatchList& L, hipStream_t s) {
    if (L.nprob < 1 || L.blocks < 1) return hipSuccess;
    if (L.wpb < 1 || L.wpb > 4) return hipErrorInvalidValue;
    switch (prec) {
        case 0: return batch_triple_t<double, double>(code, vx, L, s);
        case 1: return batch_triple_t<float, uint16_t>(code, vx, L, s);
        case 2: return batch_triple_t<float, float>(code, vx, L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ac
