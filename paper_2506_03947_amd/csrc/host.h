// Host-side internals shared by the C ABI units: api.hip (contexts, problems, the
// preconditioner stages and their drivers), solve.hip (the FGMRES outer solve),
// batch.hip (batched solves), tuner.hip (tiling control and the tile tuner) and
// cnn_api.hip (the warm-start network).  Host code only; the kernels live in the
// other .hip files behind ac_internal.h.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "alphacirc.h"
#include "ac_internal.h"
#include "tiling.h"

using ac::Geom;
using ac::kMaxEll;
using ac::kMaxShift;
using ac::Tiling;
using cplx = std::complex<double>;

// ---------------------------------------------------------------------------
// error plumbing: every ABI call returns an ac_status; fail() records the message
// that ac_last_error() reports

namespace ach {
int fail(int status, const std::string& msg);
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
}  // namespace ach

#define AC_HIP(call)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return ach::fail(AC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
    } while (0)

#define AC_TRY(call)              \
    do {                          \
        int s_ = (call);          \
        if (s_ < 0) return s_;    \
    } while (0)

// ---------------------------------------------------------------------------
// opaque types

// One stencil launch captured while a context records (batched driver): the op
// (ac::BatchOp), its kernel variant, grid and argument bytes.
struct ac_launch_rec {
    int op, ell, prec, curk, vx, wpb, blocks;
    std::vector<char> args;
};

struct ac_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    double* pinned = nullptr;  // host staging for reductions
    bool profiling = false;
    struct Pending {
        hipEvent_t a, b;
        int cls;
        double bytes;
        int launches;
    };
    std::vector<Pending> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    double ms[AC_K_COUNT] = {};
    long long launches[AC_K_COUNT] = {};
    double bytes[AC_K_COUNT] = {};
    // tiling overrides (0 = automatic): rows per wave, waves per block, points per lane
    int tile_h = 0, tile_wpb = 0, tile_vx = 0;
    // while set, stencil launch sites append records here instead of launching
    std::vector<ac_launch_rec>* rec = nullptr;
    // steady sweeps in shift groups: -1 automatic (5 or more unique shifts), 0 off, 1 on
    int shift_groups = -1;
    // two steady Chebyshev steps per sweep: 0 off, 1 on (Dirichlet grids); rows per
    // wave, points per lane, waves per block of the paired sweep (0 = automatic)
    int pairs = 1, pair_h = 0, pair_vx = 0, pair_wpb = 0;
    // three steady steps per sweep: 0 off, 1 on (where pairs are allowed); tiling as pairs
    int triples = 1, triple_h = 0, triple_vx = 0, triple_occ = 4;
    // launch-bound inner solves (P_SP) are captured on this stream and replayed as graphs
    hipStream_t cap = nullptr;
    bool graphs = true;
};

constexpr int kResidBlocks = 512;  // blocks of the warm-start residual-statistics kernel
// pinned host staging per context: reductions of up to 256 batched problems plus
// their per-step scales and masks
constexpr size_t kPinnedDoubles = 32768;

struct ac_problem {
    ac_ctx* ctx = nullptr;
    Geom g{};
    int ell = 0;
    double alpha = 0;
    int nsr = 0, nsc = 0, ns = 0;
    double* k64 = nullptr;
    float* k32 = nullptr;
    uint16_t* k16 = nullptr;
    double bounds[3][2] = {};  // per precision: mu_lo, mu_hi
    double kmin64 = 0, kmax64 = 0;
    double* rpart = nullptr;   // per-block partial sums of the warm-start residual test
    double* kblocks = nullptr; // varying diagonal blocks: l coefficient fields for calA (k64 is their mean)
    ac_cnn* cnn = nullptr;     // warm-start network (not owned)
    // sweep tiling chosen for this problem (0 = the context's setting)
    int tile_h = 0, tile_wpb = 0, tile_vx = 0;
    // multigrid hierarchy of A (AC_INNER_SP), built by ac_problem_create_multigrid
    ac::MgHierarchy mg{};
    double* mgmem = nullptr;
    // captured P_SP inner solve, valid for this workspace, step count and precision
    struct SpGraph {
        hipGraphExec_t exec = nullptr;
        const void* ws = nullptr;
        int iters = 0, prec = -1;
    } spg;
};


struct ac_cnn {
    ac_ctx* ctx = nullptr;
    char* mem = nullptr;       // one allocation for everything below
    float* w = nullptr;        // float32 master parameters
    float* g = nullptr;        // last gradient
    float* m = nullptr;        // Adam moments
    float* v = nullptr;
    uint16_t* wf = nullptr;    // bf16 forward weights [3][9][16][16]
    uint16_t* wb = nullptr;    // bf16 flipped/transposed weights for input gradients
    float* bias = nullptr;     // [3][16]
    double c0 = 0.0, c1 = 1.0; // ln kappa normalisation
    int t = 0;                 // Adam steps taken
    int fused = 1;             // inference by the fused (all layers in LDS) kernel
    int scaled = 1;            // scale each guess by its residual-minimising factor
    double accept = 1.0;       // keep a guess only if |rhat - B x0| < accept |rhat|
};

namespace ach {

// Steady Chebyshev sweeps of problems with many unique shifts run as several
// launches of the (one real, two complex shifts) kernel variant over slot groups:
// the all-shift variant needs more than 168 VGPRs at l = 10 (two waves per SIMD),
// the group variant about 110 (four waves per SIMD), which hides more memory latency
// at the price of reading kappa once per group.  Every shift is computed exactly as
// in the all-shift variant.
constexpr int kMaxGroups = 4;  // groups of (1 real, 2 complex) slots cover l <= 16

struct ProfScope {
    ac_ctx* c;
    hipEvent_t a = nullptr, b = nullptr;
    int cls;
    double bytes;
    int launches = 1;
    ProfScope(ac_ctx* ctx, int cls_, double bytes_) : c(ctx), cls(cls_), bytes(bytes_) {
        if (!c->profiling) return;
        if (!c->pool.empty()) {
            a = c->pool.back().first;
            b = c->pool.back().second;
            c->pool.pop_back();
        } else {
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
        }
        (void)hipEventRecord(a, c->stream);
    }
    ~ProfScope() {
        if (!c->profiling || !a) return;
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back({a, b, cls, bytes, launches});
    }
};

struct PrecBufs {
    char* rhat;
    char* buf[4];  // iterate buffers (the last two null for the exact and saddle-point solves)
    char* cnn;     // start of the CNN buffers or of the exact / saddle-point solve's extra buffers
};

// Per-slot sums over the grid for rhat and a guess x0 (B = A - lambda I):
// rr = |rhat|^2, bb = |B x0|^2, (cr, ci) = sum conj(B x0) rhat (zero without x0).
struct SlotStats {
    std::vector<double> rr, bb, cr, ci;
    // |rhat - c B x0|^2 for the complex factor c
    double res(int s, double c_re = 1.0, double c_im = 0.0) const {
        return rr[s] - 2.0 * (c_re * cr[s] - c_im * ci[s]) + (c_re * c_re + c_im * c_im) * bb[s];
    }
};

// Krylov workspace of one solve: basis V_0..V_m, preconditioned vectors Z_0..Z_{m-1},
// reduction partials and the preconditioner's own workspace
struct SolveWs {
    double* V[ac::kMaxBasis];
    double* Z[ac::kMaxBasis];
    double* partial;   // krylov_blocks * 72
    double* partial2;  // calA tiles
    double* red;       // 128 reduced scalars
    void* prec;
};

// ---- profiling
int harvest(ac_ctx* c);

// ---- geometry and workspace helpers (api.hip)
int slot_to_m(const ac_problem* p, int slot);
bool ranges_overlap(const void* a, const void* b, size_t bytes);
size_t block_bytes(const ac_problem* p);
Tiling sweep_tiling(const ac_problem* p);
size_t cnn_ws_bytes(const ac_problem* p);
size_t prec_ws_bytes(const ac_problem* p, int prec, int inner = AC_INNER_CHEB);
PrecBufs carve_prec(const ac_problem* p, int prec, void* ws, int inner = AC_INNER_CHEB);
size_t vec_bytes(const ac_problem* p);
size_t solve_ws_bytes(const ac_problem* p, const ac_solve_opts* o);
SolveWs carve_solve(const ac_problem* p, const ac_solve_opts* o, void* ws);
hipError_t launch_zero(double* x, long long n, hipStream_t s);
hipError_t launch_zero_int(int* x, int n, hipStream_t s);

// ---- the preconditioner and the operator (api.hip)
// Checks the options against the problem; pm receives the inner step count per slot.
int validate_opts(const ac_problem* p, const ac_solve_opts* o, std::vector<int>& pm);
// Nested-Chebyshev inner solves of every slot from rhat into z (inverse time-DFT fused).
// z is scaled by out_scale (folded into the inverse transform).
int run_cheb(ac_problem* p, int prec, const std::vector<int>& pm, char* rhat, char* const buf[4], bool warm, double* z,
             std::vector<std::pair<int, char*>>* where, double out_scale = 1.0);
// z = P^-1 (in_scale r) by the inner method of o (workspace carved by carve_prec).
int apply_prec_impl(ac_problem* p, const ac_solve_opts* o, const std::vector<int>& pm, const double* r, double* z,
                    void* ws, double in_scale, int* fallbacks = nullptr);
// Whether the inner method inside an FGMRES cycle is the plain nested Chebyshev (the
// inner modes whose in-cycle applications can start from a transform made by
// axpy_fwd_impl).
bool prec_from_rhat_ok(const ac_problem* p, const ac_solve_opts* o);
// The Gram-Schmidt update w -= sum_{q < nv} vs.s2[q] vs.v[q] fused with the forward
// transform of the new w (no input scale) into the preconditioner workspace ws; the
// per-block sums of w^2 go to partial[block * stride], *blocks of them.
int axpy_fwd_impl(ac_problem* p, const ac_solve_opts* o, const ac::VecSet& vs, int nv, double* w, void* ws,
                  double* partial, int stride, int* blocks);
// z = out_scale P^-1 applied to the transform already in ws (plain nested Chebyshev).
int apply_prec_rhat(ac_problem* p, const ac_solve_opts* o, const std::vector<int>& pm, double* z, void* ws,
                    double out_scale);
// y = calA x, or with b: y = b - calA x and per-tile partial sums of y^2.
int calA_impl(ac_problem* p, const double* x, double* y, const double* b, double* partial);
long long calA_partials(const ac_problem* p);

// ---- the warm-start network's host side (api.hip)
ac::CnnPrepArgs cnn_args(const ac_problem* p, int prec, const char* rhat);
int slot_residuals(ac_problem* p, int prec, const ac::CnnPrepArgs& a, const char* x0, SlotStats& out);
void set_rms_scales(const ac_problem* p, const SlotStats& st, ac::CnnPrepArgs& a, double* scales);
int cnn_forward_impl(ac_cnn* c, const uint16_t* x, int B, int H, int W, float* y, uint16_t* a1, uint16_t* a2,
                     hipStream_t st);
int cnn_warm_start(ac_problem* p, int prec, const char* rhat, char* x0buf, char* cws, int* fallbacks);

}  // namespace ach
