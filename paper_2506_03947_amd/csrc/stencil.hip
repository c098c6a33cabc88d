// Dispatch of the stencil kernels by the number of time blocks l; the kernels
// themselves are instantiated once per l in stencil_ell.hip.
#include <hip/hip_runtime.h>

#include "ac_internal.h"
#include "worklist.h"

namespace ac {

#define AC_DECL(L)                                                                                       \
    hipError_t sweep_ell_##L(bool final, int prec, int vx, int curk, const void* args, hipStream_t s);    \
    hipError_t fwd_ell_##L(int prec, const FwdArgs& a, hipStream_t s);                                    \
    hipError_t inv_ell_##L(int prec, const InvArgs& a, hipStream_t s);                                    \
    hipError_t calA_ell_##L(bool resid, const CalAArgs& a, hipStream_t s);                                \
    hipError_t axpy_fwd_ell_##L(int prec, const AxpyFwdArgs& a, hipStream_t s);                          \
    hipError_t batch_ell_##L(int op, int prec, int curk, int vx, const BatchList& b, hipStream_t s);
AC_DECL(2) AC_DECL(3) AC_DECL(4) AC_DECL(5) AC_DECL(6) AC_DECL(7) AC_DECL(8) AC_DECL(9) AC_DECL(10)
AC_DECL(11) AC_DECL(12) AC_DECL(13) AC_DECL(14) AC_DECL(15) AC_DECL(16)
#undef AC_DECL

#define AC_SWITCH(EXPR_OF_L)                                                                  \
    switch (ell) {                                                                            \
        case 2: return EXPR_OF_L(2);                                                          \
        case 3: return EXPR_OF_L(3);                                                          \
        case 4: return EXPR_OF_L(4);                                                          \
        case 5: return EXPR_OF_L(5);                                                          \
        case 6: return EXPR_OF_L(6);                                                          \
        case 7: return EXPR_OF_L(7);                                                          \
        case 8: return EXPR_OF_L(8);                                                          \
        case 9: return EXPR_OF_L(9);                                                          \
        case 10: return EXPR_OF_L(10);                                                        \
        case 11: return EXPR_OF_L(11);                                                        \
        case 12: return EXPR_OF_L(12);                                                        \
        case 13: return EXPR_OF_L(13);                                                        \
        case 14: return EXPR_OF_L(14);                                                        \
        case 15: return EXPR_OF_L(15);                                                        \
        case 16: return EXPR_OF_L(16);                                                        \
        default: return hipErrorInvalidValue;                                                 \
    }

static int sweep_vx(int prec, const void* args) {
    return prec == 0 ? static_cast<const SweepArgs<double>*>(args)->t.vx
                     : static_cast<const SweepArgs<float>*>(args)->t.vx;
}

hipError_t launch_cheb_step(int ell, int prec, int curk, const void* args, hipStream_t s) {
    const int vx = sweep_vx(prec, args);
#define AC_X(L) sweep_ell_##L(false, prec, vx, curk, args, s)
    AC_SWITCH(AC_X)
#undef AC_X
}

hipError_t launch_cheb_final(int ell, int prec, int curk, const void* args, hipStream_t s) {
    const int vx = sweep_vx(prec, args);
#define AC_X(L) sweep_ell_##L(true, prec, vx, curk, args, s)
    AC_SWITCH(AC_X)
#undef AC_X
}

hipError_t launch_tdft_fwd(int ell, int prec, const FwdArgs& a, hipStream_t s) {
#define AC_X(L) fwd_ell_##L(prec, a, s)
    AC_SWITCH(AC_X)
#undef AC_X
}

hipError_t launch_tdft_inv(int ell, int prec, const InvArgs& a, hipStream_t s) {
#define AC_X(L) inv_ell_##L(prec, a, s)
    AC_SWITCH(AC_X)
#undef AC_X
}

hipError_t launch_apply_calA(int ell, bool resid, const CalAArgs& a, hipStream_t s) {
#define AC_X(L) calA_ell_##L(resid, a, s)
    AC_SWITCH(AC_X)
#undef AC_X
}

hipError_t launch_axpy_fwd(int ell, int prec, const AxpyFwdArgs& a, hipStream_t s) {
    if (a.nv < 1 || a.nv > 32) return hipErrorInvalidValue;
#define AC_X(L) axpy_fwd_ell_##L(prec, a, s)
    AC_SWITCH(AC_X)
#undef AC_X
}

hipError_t launch_batch(int op, int ell, int prec, int curk, int vx, const BatchList& b, hipStream_t s) {
    if (b.nprob > kListMax) return hipErrorInvalidValue;
    if (op == BOP_TRIPLE) return launch_batch_triple(prec, curk, vx, b, s);  // not specialised by l
    if (op == BOP_PAIR) return launch_batch_pair(prec, vx, b, s);
#define AC_X(L) batch_ell_##L(op, prec, curk, vx, b, s)
    AC_SWITCH(AC_X)
#undef AC_X
}

}  // namespace ac
