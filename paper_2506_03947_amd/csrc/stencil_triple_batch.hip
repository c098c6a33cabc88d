// Batched (work-list) launches of the three-step shifted-Chebyshev sweep over many
// problems of uneven size (the device body is in stencil_triple.h): every entry of a
// list has the same number of shift groups (L.wpb waves per workgroup).
#include "stencil_triple.h"

namespace ac {
namespace {

template <typename R, typename KS>
hipError_t batch_triple_t(int code, int vx, const BatchList& L, hipStream_t s) {
    const bool first = (code & 2) != 0;
    const dim3 grid(list_grid(L.blocks, L.nprob, L.wpb)), block(L.wpb * kWave);
    if (vx == 2) {
        if (first) hipLaunchKernelGGL((cheb_triple_batch_kernel<R, KS, 2, true>), grid, block, 0, s, L);
        else hipLaunchKernelGGL((cheb_triple_batch_kernel<R, KS, 2, false>), grid, block, 0, s, L);
    } else if (vx == 1) {
        if (first) hipLaunchKernelGGL((cheb_triple_batch_kernel<R, KS, 1, true>), grid, block, 0, s, L);
        else hipLaunchKernelGGL((cheb_triple_batch_kernel<R, KS, 1, false>), grid, block, 0, s, L);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch_triple(int prec, int code, int vx, const BatchList& L, hipStream_t s) {
    if (L.nprob < 1 || L.blocks < 1) return hipSuccess;
    if (L.wpb < 1 || L.wpb > kMaxTripleGroups) return hipErrorInvalidValue;
    switch (prec) {
        case 0: return batch_triple_t<double, double>(code, vx, L, s);
        case 1: return batch_triple_t<float, uint16_t>(code, vx, L, s);
        case 2: return batch_triple_t<float, float>(code, vx, L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ac
