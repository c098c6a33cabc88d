// Instantiates the stencil kernels for one number of time blocks l = AC_ELL.
// The build compiles this file once per l in [2, 16] (-DAC_ELL=l) so that the
// several hundred kernel variants compile in parallel.
#include "stencil_kernels.h"

#ifndef AC_ELL
#error "compile with -DAC_ELL=<l>"
#endif

namespace ac {
namespace {

template <typename R, typename KS, int VX, bool CUR_RHAT, bool FINAL, bool PER>
hipError_t launch_sweep_t(const SweepArgs<R>& a, hipStream_t s) {
    hipLaunchKernelGGL((cheb_sweep_kernel<R, KS, AC_ELL, VX, CUR_RHAT, FINAL, PER>), dim3(a.t.blocks),
                       dim3(a.t.wpb * kWave), 0, s, a);
    return hipGetLastError();
}

template <typename R, typename KS, bool FINAL>
hipError_t sweep_by_kind(int vx, int curk, const void* args, hipStream_t s) {
    const SweepArgs<R>& a = *static_cast<const SweepArgs<R>*>(args);
    const bool rh = (curk == SRC_RHAT);
    if (a.g.periodic) {
        if (vx != 1) return hipErrorInvalidValue;
        return rh ? launch_sweep_t<R, KS, 1, true, FINAL, true>(a, s) : launch_sweep_t<R, KS, 1, false, FINAL, true>(a, s);
    }
    if (vx == 2)
        return rh ? launch_sweep_t<R, KS, 2, true, FINAL, false>(a, s) : launch_sweep_t<R, KS, 2, false, FINAL, false>(a, s);
    return rh ? launch_sweep_t<R, KS, 1, true, FINAL, false>(a, s) : launch_sweep_t<R, KS, 1, false, FINAL, false>(a, s);
}

template <bool FINAL>
hipError_t sweep_by_prec(int prec, int vx, int curk, const void* args, hipStream_t s) {
    switch (prec) {
        case 0: return sweep_by_kind<double, double, FINAL>(vx, curk, args, s);
        case 1: return sweep_by_kind<float, uint16_t, FINAL>(vx, curk, args, s);
        case 2: return sweep_by_kind<float, float, FINAL>(vx, curk, args, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

#define AC_CAT2(a, b) a##b
#define AC_CAT(a, b) AC_CAT2(a, b)

hipError_t AC_CAT(sweep_ell_, AC_ELL)(bool final, int prec, int vx, int curk, const void* args, hipStream_t s) {
    return final ? sweep_by_prec<true>(prec, vx, curk, args, s) : sweep_by_prec<false>(prec, vx, curk, args, s);
}

hipError_t AC_CAT(fwd_ell_, AC_ELL)(int prec, const FwdArgs& a, hipStream_t s) {
    constexpr int ELL = AC_ELL;
    int vx, blocks;
    fwd_geometry(a.n, vx, blocks);
    if (prec == 0) {
        if (vx == 2) hipLaunchKernelGGL((tdft_fwd_kernel<double, ELL, 2>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((tdft_fwd_kernel<double, ELL, 1>), dim3(blocks), dim3(256), 0, s, a);
    } else {
        if (vx == 2) hipLaunchKernelGGL((tdft_fwd_kernel<float, ELL, 2>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((tdft_fwd_kernel<float, ELL, 1>), dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t AC_CAT(inv_ell_, AC_ELL)(int prec, const InvArgs& a, hipStream_t s) {
    constexpr int ELL = AC_ELL;
    const int vx = (a.n % 2 == 0) ? 2 : 1;
    const long long threads = (a.n + vx - 1) / vx;
    const int blocks = static_cast<int>((threads + 255) / 256);
    if (prec == 0) {
        if (vx == 2) hipLaunchKernelGGL((tdft_inv_kernel<double, ELL, 2>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((tdft_inv_kernel<double, ELL, 1>), dim3(blocks), dim3(256), 0, s, a);
    } else {
        if (vx == 2) hipLaunchKernelGGL((tdft_inv_kernel<float, ELL, 2>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((tdft_inv_kernel<float, ELL, 1>), dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// The Gram-Schmidt update fused with the forward transform: one point per lane on
// odd grids, two otherwise; the basis bound NVB = 8 or 32.
hipError_t AC_CAT(axpy_fwd_ell_, AC_ELL)(int prec, const AxpyFwdArgs& a, hipStream_t s) {
    constexpr int ELL = AC_ELL;
    const int vx = (a.f.n % 2 == 0) ? 2 : 1;
    const int blocks = axpy_fwd_blocks(a.f.n);
    const bool small = a.nv <= 8;
#define AC_AF(R, VX, NVB) hipLaunchKernelGGL((axpy_fwd_kernel<R, ELL, VX, NVB>), dim3(blocks), dim3(256), 0, s, a)
    if (prec == 0) {
        if (vx == 2) { if (small) AC_AF(double, 2, 8); else AC_AF(double, 2, 32); }
        else { if (small) AC_AF(double, 1, 8); else AC_AF(double, 1, 32); }
    } else {
        if (vx == 2) { if (small) AC_AF(float, 2, 8); else AC_AF(float, 2, 32); }
        else { if (small) AC_AF(float, 1, 8); else AC_AF(float, 1, 32); }
    }
#undef AC_AF
    return hipGetLastError();
}

hipError_t AC_CAT(calA_ell_, AC_ELL)(bool resid, const CalAArgs& a, hipStream_t s) {
    constexpr int ELL = AC_ELL;
    const dim3 grid(a.t.blocks), block(a.t.wpb * kWave);
    if (calA_strips(a.g)) {
        if (a.t.vx == 2) {
            if (resid) hipLaunchKernelGGL((apply_calA_strip_kernel<ELL, 2, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((apply_calA_strip_kernel<ELL, 2, false>), grid, block, 0, s, a);
        } else {
            if (resid) hipLaunchKernelGGL((apply_calA_strip_kernel<ELL, 1, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((apply_calA_strip_kernel<ELL, 1, false>), grid, block, 0, s, a);
        }
        return hipGetLastError();
    }
    if (a.t.vx == 2) {
        if (resid) hipLaunchKernelGGL((apply_calA_kernel<ELL, 2, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((apply_calA_kernel<ELL, 2, false>), grid, block, 0, s, a);
    } else {
        if (resid) hipLaunchKernelGGL((apply_calA_kernel<ELL, 1, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((apply_calA_kernel<ELL, 1, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace ac
