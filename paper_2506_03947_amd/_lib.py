"""ctypes declarations for libalphacirc.so (include/alphacirc.h).

Loading fails loudly: there is no CPU fallback.  Build the library with
``python -m paper_2506_03947_amd.build``.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libalphacirc.so")

AC_OK = 0
AC_NOT_CONVERGED = 1
AC_ERR_ARG = -1
AC_ERR_ALPHA = -2
AC_ERR_BOUNDS = -3
AC_ERR_HIP = -4
AC_ERR_WORKSPACE = -5
AC_ERR_NONFINITE = -6
AC_ERR_UNSUPPORTED = -7

AC_BC_DIRICHLET = 0
AC_BC_PERIODIC = 1

AC_PREC_FP64 = 0
AC_PREC_MIXED_BF16K = 1
AC_PREC_MIXED_FP32K = 2

AC_INNER_CHEB = 0
AC_INNER_CHEB_CNN = 1
AC_INNER_CHEB_CNN_CYCLE = 2
AC_INNER_EXACT = 3
AC_INNER_SP = 4
AC_INNER_CHEB_CNN_MR = 5
AC_NOALLOC_SCRATCH_BYTES = 64 << 20  # fixed device scratch of ac_apply_prec_noalloc

AC_OUTER_FGMRES = 0
AC_OUTER_CHEBYSHEV = 1

AC_K_TDFT_FWD = 0
AC_K_CHEB_STEP = 1
AC_K_CHEB_FINAL = 2
AC_K_APPLY_CALA = 3
AC_K_KRYLOV = 4
AC_K_CNN = 5
AC_K_CHEB_FIRST = 6
AC_K_EXACT = 7
AC_K_SADDLE = 8
AC_K_CHEB_PAIR = 9
AC_K_CHEB_TRIPLE = 10
AC_K_COUNT = 11
KERNEL_CLASS_NAMES = ["tdft_fwd", "cheb_step", "cheb_final", "apply_calA", "krylov", "cnn", "cheb_first", "exact",
                      "saddle", "cheb_pair", "cheb_triple"]


class ac_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("bc", C.c_int)]


class ac_bounds(C.Structure):
    _fields_ = [("mu_lo", C.c_double), ("mu_hi", C.c_double)]


class ac_solve_opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int),
        ("inner", C.c_int),
        ("p_per_shift", C.POINTER(C.c_int)),
        ("p_uniform", C.c_int),
        ("tol", C.c_double),
        ("restart_m", C.c_int),
        ("max_outer", C.c_int),
        ("outer", C.c_int),
    ]


class ac_solve_info(C.Structure):
    _fields_ = [
        ("outer_iters", C.c_int),
        ("restarts", C.c_int),
        ("matvecs_A", C.c_longlong),
        ("rel_residual_true", C.c_double),
        ("seconds", C.c_double),
        ("cnn_fallbacks", C.c_int),
        ("reserved", C.c_int),
        ("orth_loss", C.c_double),
    ]


# name -> (restype, argtypes); every entry is an exported symbol of the library
_VP = C.c_void_p
_I = C.c_int
_D = C.c_double
_SZ = C.c_size_t
SIGNATURES = {
    "ac_status_string": (C.c_char_p, [_I]),
    "ac_last_error": (C.c_char_p, []),
    "ac_ctx_create": (_I, [_I, _VP, C.POINTER(_VP)]),
    "ac_ctx_destroy": (_I, [_VP]),
    "ac_ctx_set_stream": (_I, [_VP, _VP]),
    "ac_ctx_set_profiling": (_I, [_VP, _I]),
    "ac_ctx_kernel_stats": (_I, [_VP, C.POINTER(_D), C.POINTER(C.c_longlong), C.POINTER(_D)]),
    "ac_ctx_reset_stats": (_I, [_VP]),
    "ac_ctx_set_tiling": (_I, [_VP, _I, _I, _I]),
    "ac_problem_create": (_I, [_VP, C.POINTER(ac_grid), _VP, _I, _D, C.POINTER(ac_bounds), C.POINTER(_VP)]),
    "ac_problem_create_blocks": (_I, [_VP, C.POINTER(ac_grid), _VP, _I, _D, C.POINTER(ac_bounds), C.POINTER(_VP)]),
    "ac_problem_destroy": (_I, [_VP]),
    "ac_problem_create_multigrid": (_I, [_VP]),
    "ac_ctx_set_graphs": (_I, [_VP, _I]),
    "ac_mg_workspace_size": (_I, [_VP, _I, C.POINTER(_SZ)]),
    "ac_mg_vcycle": (_I, [_VP, _I, C.POINTER(_D), _VP, _VP, _VP, _SZ]),
    "ac_spectral_bounds": (_I, [_VP, C.POINTER(_D), C.POINTER(_D)]),
    "ac_problem_dims": (_I, [_VP, C.POINTER(C.c_longlong), C.POINTER(_I), C.POINTER(_I)]),
    "ac_alloc_nc2": (_I, [_VP, _D, C.POINTER(_I)]),
    "ac_alloc_nc1": (_I, [_VP, _D, C.POINTER(_I)]),
    "ac_prec_workspace_size": (_I, [_VP, C.POINTER(ac_solve_opts), C.POINTER(_SZ)]),
    "ac_solve_workspace_size": (_I, [_VP, C.POINTER(ac_solve_opts), C.POINTER(_SZ)]),
    "ac_apply_A": (_I, [_VP, _VP, _VP]),
    "ac_apply_prec": (_I, [_VP, C.POINTER(ac_solve_opts), _VP, _VP, _VP, _SZ]),
    "ac_apply_prec_noalloc": (_I, [_VP, C.POINTER(ac_solve_opts), _VP, _VP]),
    "ac_stream_bandwidth": (_I, [_VP, _I, _I, _VP, _SZ, _I, C.POINTER(_D)]),
    "ac_spectral_offsets": (_I, [_VP, _I, C.POINTER(C.c_longlong)]),
    "ac_tdft_forward": (_I, [_VP, _I, _VP, _VP]),
    "ac_shifted_cheb": (_I, [_VP, C.POINTER(ac_solve_opts), _VP, _VP, _VP, _VP, _SZ]),
    "ac_tdft_inverse": (_I, [_VP, _I, _VP, _VP]),
    "ac_solve": (_I, [_VP, C.POINTER(ac_solve_opts), _VP, _VP, _VP, _SZ, C.POINTER(ac_solve_info)]),
    "ac_batch_workspace_size": (_I, [_VP, _I, C.POINTER(_VP), C.POINTER(ac_solve_opts), C.POINTER(_SZ)]),
    "ac_batch_solve": (_I, [_VP, _I, C.POINTER(_VP), C.POINTER(ac_solve_opts), C.POINTER(_VP), C.POINTER(_VP), _VP,
                            _SZ, C.POINTER(ac_solve_info)]),
    "ac_solve_record": (_I, [_VP, C.POINTER(ac_solve_opts), _VP, _VP, _VP, _SZ, C.POINTER(ac_solve_info), _VP, _I,
                             C.POINTER(_I)]),
    "ac_cnn_param_count": (_I, []),
    "ac_cnn_create": (_I, [_VP, C.POINTER(_VP)]),
    "ac_cnn_destroy": (_I, [_VP]),
    "ac_cnn_set_params": (_I, [_VP, C.POINTER(C.c_float), _D, _D]),
    "ac_cnn_get_params": (_I, [_VP, C.POINTER(C.c_float), C.POINTER(_D), C.POINTER(_D)]),
    "ac_cnn_workspace_size": (_I, [_I, _I, _I, C.POINTER(_SZ)]),
    "ac_cnn_forward": (_I, [_VP, _VP, _I, _I, _I, _VP, _VP, _SZ]),
    "ac_cnn_grad": (_I, [_VP, _VP, _VP, _VP, _I, _I, _I, _I, _VP, _SZ, C.POINTER(_D), C.POINTER(C.c_float)]),
    "ac_cnn_grad_residual": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _I, _I, _I, _I, _VP, _SZ, C.POINTER(_D),
                                  C.POINTER(C.c_float)]),
    "ac_problem_shifts": (_I, [_VP, C.POINTER(_D)]),
    "ac_problem_set_tiling": (_I, [_VP, _I, _I, _I]),
    "ac_ctx_set_shift_groups": (_I, [_VP, _I]),
    "ac_ctx_set_step_pairs": (_I, [_VP, _I, _I, _I, _I]),
    "ac_ctx_set_step_triples": (_I, [_VP, _I, _I, _I, _I]),
    "ac_tune_tiling": (_I, [_VP, _I, C.c_char_p, _VP, _SZ, C.POINTER(C.c_int), C.POINTER(_D)]),
    "ac_cnn_adam_step": (_I, [_VP, _D, _D, _D, _D]),
    "ac_cnn_make_inputs": (_I, [_VP, _VP, _I, _VP, _VP, C.POINTER(_D), _VP]),
    "ac_problem_attach_cnn": (_I, [_VP, _VP]),
    "ac_shifted_residual": (_I, [_VP, _I, _VP, _VP, C.POINTER(_D)]),
    "ac_cnn_guess_workspace_size": (_I, [_VP, C.POINTER(_SZ)]),
    "ac_cnn_guess": (_I, [_VP, _I, _VP, _VP, _VP, _SZ, C.POINTER(_I)]),
    "ac_cnn_set_guess_policy": (_I, [_VP, _I, _D]),
    "ac_cnn_set_inference": (_I, [_VP, _I]),
}

_lib = None


def load() -> C.CDLL:
    """Load libalphacirc.so once; raise if it is missing or lacks a symbol."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2506_03947_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class AlphacircError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.ac_last_error().decode()
        super().__init__(f"{where}: {lib.ac_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise AlphacircError(status, where)
    return status
