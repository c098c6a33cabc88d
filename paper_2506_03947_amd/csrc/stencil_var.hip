// Launcher of the all-at-once operator with varying diagonal blocks (one coefficient
// field per time block); independent of l, so compiled once.
#include "stencil_kernels.h"

namespace ac {

hipError_t launch_apply_calA_var(int ell, bool resid, const CalAArgs& a, hipStream_t s) {
    if (ell < 1) return hipErrorInvalidValue;
    const dim3 grid(a.t.blocks, ell), block(a.t.wpb * kWave);
    if (a.t.vx == 2) {
        if (resid) hipLaunchKernelGGL((apply_calA_var_kernel<2, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((apply_calA_var_kernel<2, false>), grid, block, 0, s, a);
    } else {
        if (resid) hipLaunchKernelGGL((apply_calA_var_kernel<1, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((apply_calA_var_kernel<1, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace ac
