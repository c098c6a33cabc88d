// Launches of the three-step shifted-Chebyshev sweep for one problem (the device body
// is in stencil_triple.h).
#include "stencil_triple.h"

namespace ac {
namespace {

template <typename R, typename KS, int VX, bool FIRST>
hipError_t triple_by_kind(const TripleArgs<R>& a, hipStream_t s) {
    const dim3 grid(a.t.blocks), block(a.t.wpb * kWave);
    if (a.kind == 0) hipLaunchKernelGGL((cheb_triple_kernel<R, KS, VX, 2, 1, FIRST>), grid, block, 0, s, a);
    else if (a.kind == 1) hipLaunchKernelGGL((cheb_triple_kernel<R, KS, VX, 1, 2, FIRST>), grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R, typename KS>
hipError_t triple_launch_t(const void* args, hipStream_t s) {
    const TripleArgs<R>& a = *static_cast<const TripleArgs<R>*>(args);
    if (a.g.periodic || a.t.blocks <= 0 || a.t.wpb < 1 || a.t.wpb > 4 || a.g.nx < 4) return hipErrorInvalidValue;
    if (a.t.vx == 2 && a.g.nx % 2 != 0) return hipErrorInvalidValue;
    if (a.t.vx == 2) return a.first ? triple_by_kind<R, KS, 2, true>(a, s) : triple_by_kind<R, KS, 2, false>(a, s);
    if (a.t.vx == 1) return a.first ? triple_by_kind<R, KS, 1, true>(a, s) : triple_by_kind<R, KS, 1, false>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_cheb_triple(int prec, const void* args, hipStream_t s) {
    switch (prec) {
        case 0: return triple_launch_t<double, double>(args, s);
        case 1: return triple_launch_t<float, uint16_t>(args, s);
        case 2: return triple_launch_t<float, float>(args, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ac
