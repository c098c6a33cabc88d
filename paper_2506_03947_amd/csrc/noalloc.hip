// P_NC^{-1} r for callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid hipMalloc): the workspace of ac_apply_prec comes
// from one fixed array in device memory instead of the caller.
//
// The array is a file-scope __device__ object of this translation unit; every GPU the
// library runs on holds its own copy until the process ends.  In host code its name is
// only a stand-in for the symbol, so its device address is looked up once per device
// with hipGetSymbolAddress (from ac_ctx_create, that device current) and only that
// address is ever handed to kernels.  Every call on one device shares the array and
// leaves the last call's contents in it: calls that overlap on one device race.  The
// preconditioner reads none of its workspace before writing it, so nothing is cleared.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "alphacirc.h"
#include "ac_internal.h"

namespace {

constexpr size_t kScratchBytes = AC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

void* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

}  // namespace

namespace ac {

int noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return set_error(AC_ERR_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return AC_OK;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void* ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
        return set_error(AC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = ptr;
    return AC_OK;
}

}  // namespace ac

int ac_apply_prec_noalloc(ac_problem* p, const ac_solve_opts* opts, const double* r, double* z) {
    if (!p || !opts || !r || !z) return ac::set_error(AC_ERR_ARG, "NULL argument");
    if (opts->inner != AC_INNER_CHEB)
        return ac::set_error(AC_ERR_UNSUPPORTED, "ac_apply_prec_noalloc runs the plain nested-Chebyshev inner solve only");
    size_t need = 0;
    const int s = ac_prec_workspace_size(p, opts, &need);
    if (s < 0) return s;
    if (need > kScratchBytes)
        return ac::set_error(AC_ERR_WORKSPACE, "problem needs " + std::to_string(need) + " workspace bytes, above the " +
                                                   std::to_string(kScratchBytes) + "-byte fixed scratch");
    void* ptr = scratch_of(ac::problem_device(p));
    if (!ptr) return ac::set_error(AC_ERR_HIP, "fixed scratch not set up for this device");
    return ac_apply_prec(p, opts, r, z, ptr, kScratchBytes);
}
