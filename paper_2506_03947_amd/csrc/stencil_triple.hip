// Launches of the three-step shifted-Chebyshev sweep for one problem (the device body
// is in stencil_triple.h): one launch per block of three steps over every shift group,
// a workgroup per tile with one wave per group.
#include "stencil_triple.h"

namespace ac {
namespace {

template <typename R, typename KS>
hipError_t triple_launch_t(const void* args, hipStream_t s) {
    const TripleArgs<R>& a = *static_cast<const TripleArgs<R>*>(args);
    if (a.g.periodic || a.t.blocks <= 0 || a.g.nx < 4) return hipErrorInvalidValue;
    if (a.ngroups < 1 || a.ngroups > kMaxTripleGroups || a.t.wpb != a.ngroups) return hipErrorInvalidValue;
    if (a.t.tiles != a.t.blocks) return hipErrorInvalidValue;
    if (a.t.vx == 2 && a.g.nx % 2 != 0) return hipErrorInvalidValue;
    const dim3 grid(a.t.blocks), block(a.ngroups * kWave);
    if (a.t.vx == 2) {
        if (a.first) hipLaunchKernelGGL((cheb_triple_kernel<R, KS, 2, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cheb_triple_kernel<R, KS, 2, false>), grid, block, 0, s, a);
    } else if (a.t.vx == 1) {
        if (a.first) hipLaunchKernelGGL((cheb_triple_kernel<R, KS, 1, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cheb_triple_kernel<R, KS, 1, false>), grid, block, 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
