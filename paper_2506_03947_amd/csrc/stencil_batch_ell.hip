// Instantiates the batched (work-list) stencil launches for one number of time
// blocks l = AC_ELL; compiled once per l in [2, 16] (-DAC_ELL=l), beside the
// single-problem variants of stencil_ell.hip.
#include "stencil_kernels.h"

#ifndef AC_ELL
#error "compile with -DAC_ELL=<l>"
#endif

namespace ac {
namespace {

template <typename R, typename KS, int VX, bool FINAL>
hipError_t sweep_batch_t(int curk, const BatchList& L, hipStream_t s) {
    const dim3 grid(list_grid(L.blocks, L.nprob, L.wpb)), block(L.wpb * kWave);
    if (curk == SRC_RHAT)
        hipLaunchKernelGGL((cheb_sweep_batch_kernel<R, KS, AC_ELL, VX, true, FINAL>), grid, block, 0, s, L);
    else
        hipLaunchKernelGGL((cheb_sweep_batch_kernel<R, KS, AC_ELL, VX, false, FINAL>), grid, block, 0, s, L);
    return hipGetLastError();
}

template <typename R, typename KS, bool FINAL>
hipError_t sweep_batch_vx(int vx, int curk, const BatchList& L, hipStream_t s) {
    return vx == 2 ? sweep_batch_t<R, KS, 2, FINAL>(curk, L, s) : sweep_batch_t<R, KS, 1, FINAL>(curk, L, s);
}

template <bool FINAL>
hipError_t sweep_batch_prec(int prec, int vx, int curk, const BatchList& L, hipStream_t s) {
    switch (prec) {
        case 0: return sweep_batch_vx<double, double, FINAL>(vx, curk, L, s);
        case 1: return sweep_batch_vx<float, uint16_t, FINAL>(vx, curk, L, s);
        case 2: return sweep_batch_vx<float, float, FINAL>(vx, curk, L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

#define AC_CAT2(a, b) a##b
#define AC_CAT(a, b) AC_CAT2(a, b)

hipError_t AC_CAT(batch_ell_, AC_ELL)(int op, int prec, int curk, int vx, const BatchList& L, hipStream_t s) {
    if (L.nprob < 1 || L.blocks < 1) return hipSuccess;
    if (vx != 1 && vx != 2) return hipErrorInvalidValue;
    switch (op) {
        case BOP_STEP: return sweep_batch_prec<false>(prec, vx, curk, L, s);
        case BOP_FINAL: return sweep_batch_prec<true>(prec, vx, curk, L, s);
        case BOP_FWD: {
            const dim3 grid(list_grid(L.blocks, L.nprob, 4)), block(256);
            if (prec == 0) {
                if (vx == 2) hipLaunchKernelGGL((tdft_fwd_batch_kernel<double, AC_ELL, 2>), grid, block, 0, s, L);
                else hipLaunchKernelGGL((tdft_fwd_batch_kernel<double, AC_ELL, 1>), grid, block, 0, s, L);
            } else {
                if (vx == 2) hipLaunchKernelGGL((tdft_fwd_batch_kernel<float, AC_ELL, 2>), grid, block, 0, s, L);
                else hipLaunchKernelGGL((tdft_fwd_batch_kernel<float, AC_ELL, 1>), grid, block, 0, s, L);
            }
            return hipGetLastError();
        }
        case BOP_CALA:
        case BOP_CALA_RES: {  // residual form: y = b - calA x with per-tile partial sums of y^2
            // curk: 1 = overlapping strips, 0 = halo loads (the members' shared form)
            const dim3 grid(list_grid(L.blocks, L.nprob, L.wpb)), block(L.wpb * kWave);
#define AC_CALA_B(VX, R, S) hipLaunchKernelGGL((apply_calA_batch_kernel<AC_ELL, VX, R, S>), grid, block, 0, s, L)
            const bool res = op == BOP_CALA_RES;
            if (curk == 1) {
                if (vx == 2) { if (res) AC_CALA_B(2, true, true); else AC_CALA_B(2, false, true); }
                else { if (res) AC_CALA_B(1, true, true); else AC_CALA_B(1, false, true); }
            } else {
                if (vx == 2) { if (res) AC_CALA_B(2, true, false); else AC_CALA_B(2, false, false); }
                else { if (res) AC_CALA_B(1, true, false); else AC_CALA_B(1, false, false); }
            }
#undef AC_CALA_B
            return hipGetLastError();
        }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ac
