// Internal declarations shared by the alphacirc HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

struct ac_problem;  // the ABI's opaque problem and context (alphacirc.h)
struct ac_ctx;

namespace ac {

constexpr int kMaxEll = 16;
constexpr int kMaxShift = kMaxEll / 2 + 1;  // unique shifts l_s = floor(l/2) + 1
constexpr int kWave = 64;                   // CDNA wavefront
constexpr int kMaxBasis = 33;               // FGMRES(32): V_0..V_32

// Grid geometry.  dim 1 has faces in x only.
struct Geom {
    int nx, ny;
    int dim;
    int periodic;
    long long n;
};

// Marching-stencil tiling: every wave owns a strip of 64*vx columns and a chunk
// of h rows, and walks the chunk row by row keeping three rows in registers.
struct Tiling {
    int vx;         // consecutive x points per lane (1 or 2)
    int h;          // rows per wave
    int wpb;        // waves per block
    int nsx, ncy;   // strips in x, chunks in y
    long long tiles;
    int blocks;
};

// Where a Chebyshev operand comes from.
enum Src : int {
    SRC_BUF = 0,      // an iterate buffer
    SRC_RHAT = 1,     // x_1 = rhat / theta (zero initial guess, never stored)
    SRC_ZERO = 2,     // x_0 = 0
    SRC_COMPUTE = 3,  // (final sweep) computed in this launch
};

// Per-shift Chebyshev data for one sweep.  Shift slot order: real shifts first
// (m = 0, then m = l/2 for even l), then complex shifts m = 1..ceil(l/2)-1.
template <typename R>
struct ShiftCoef {
    R lam_re[kMaxShift], lam_im[kMaxShift];  // lambda_m
    R a_re[kMaxShift], a_im[kMaxShift];      // rho_k rho_{k-1}  (momentum)
    R c_re[kMaxShift], c_im[kMaxShift];      // 2 rho_k / delta  (residual weight)
    R s_re[kMaxShift], s_im[kMaxShift];      // 1 / theta        (x_1 = rhat / theta)
};

template <typename R>
struct SweepArgs {
    Geom g;
    Tiling t;
    const void* kappa;  // storage type depends on the precision
    ShiftCoef<R> cf;
    int src[kMaxShift];        // SRC_COMPUTE, or (final sweep) SRC_RHAT / SRC_BUF for finished shifts
    int fbuf[kMaxShift];       // final sweep, SRC_BUF: finished iterate in bufs[fbuf]
    unsigned soff[kMaxShift];  // slot offset (elements of R) inside every spectral buffer
    int prevk;                 // kind of x_{k-1}: SRC_ZERO / SRC_RHAT / SRC_BUF
    const R* rhat;             // spectral buffers (identical layouts)
    const R* cur;              // x_k
    R* out;                    // x_{k+1} (may be the buffer of x_{k-1}: each lane reads before it writes)
    const R* prev;             // x_{k-1} (when a buffer)
    const R* bufs[4];          // iterate buffers (final sweep: finished iterates)
    // inverse transform (final sweep only)
    double ginv[kMaxEll];             // 1 / (l * alpha^{k/l})
    double cw[kMaxEll], sw[kMaxEll];  // cos / sin (2 pi j / l)
    double* z;
};

// Two consecutive steady Chebyshev steps (x_{k+1} and x_{k+2}) in one sweep, for one
// group of shift slots: slot 0 real, slots 1 and 2 complex (as the l = 5 sweep).
// Tiling: strips of 64*vx computed columns at a stride of 64*vx - 2 (the two edge
// columns of a strip only feed the second step of its inner columns).
template <typename R>
struct PairArgs {
    Geom g;
    Tiling t;
    const void* kappa;
    ShiftCoef<R> cf[2];  // steps k and k+1
    int comp[3];         // slot computes (else skipped)
    unsigned soff[3];    // slot offset (elements of R) inside every spectral buffer
    const R* rhat;
    const R* cur;        // x_k
    const R* prev;       // x_{k-1}
    R* out1;             // x_{k+1}
    R* out2;             // x_{k+2}
    unsigned bytes;      // bytes of each spectral buffer (below 2^31)
};

// Three consecutive steady Chebyshev steps (x_{k+1} kept in registers, x_{k+2} and
// x_{k+3} written) in one sweep, for one group: up to two real shift slots (kind 0) or
// one complex slot (kind 1).  Strips of 64*vx computed columns advance by 64*vx - 4.
// One shift group of a three-step block: one complex shift or up to two real shifts
// (slots 0, 1), with the coefficients of steps k, k+1, k+2 (index t) in the folded form
// x_{k+1} = g x_k - a x_{k-1} + c (rhat - A' x_k), A' = A without the shift,
// g = 1 + a + c lambda (the first block of a zero-guess solve scales them for
// x_1 = rhat / theta).
template <typename R>
struct TripleGroup {
    int kind;            // 0: real slots, 1: one complex slot
    int comp[2];         // slot computes (else skipped)
    unsigned soff[2];    // slot offset (elements of R) inside every spectral buffer
    R g_re[3][2], g_im[3][2];
    R a_re[3][2], a_im[3][2];
    R c_re[3][2], c_im[3][2];
};

// Real shifts share one group, every complex shift has its own: l <= 16 gives at most
// one real group and seven complex ones.
constexpr int kMaxTripleGroups = 8;

template <typename R>
struct TripleArgs {
    Geom g;
    Tiling t;            // one tile per workgroup, one wave per group (t.wpb = ngroups)
    const void* kappa;
    const R* rhat;
    const R* cur;        // x_k
    const R* prev;       // x_{k-1}
    R* outz;             // x_{k+2}
    R* outw;             // x_{k+3}
    unsigned bytes;      // bytes of each spectral buffer (below 2^31)
    int first;           // steps 1..3 from a zero guess: x_1 = rhat / theta (never stored), x_0 = 0
    int ngroups;
    TripleGroup<R> grp[kMaxTripleGroups];
};

struct FwdArgs {
    long long n;
    double gam[kMaxEll];              // input scale * alpha^{k/l}
    double cw[kMaxEll], sw[kMaxEll];  // cos / sin (2 pi j / l)
    const double* r;
    void* rhat[kMaxShift];            // slot order as ShiftCoef
};

// Gram-Schmidt update of the newest Krylov vector fused with the forward transform
// (axpy_fwd_kernel): w -= sum_{q < nv} c[q] v[q], then f's transform of w into f.rhat
// (f.r unused), per-block sums of w^2 at partial[block * stride].
struct AxpyFwdArgs {
    FwdArgs f;
    const double* v[kMaxBasis];
    double c[kMaxBasis];
    int nv;
    int stride;
    double* w;
    double* partial;
};

struct InvArgs {
    long long n;
    double ginv[kMaxEll];
    double cw[kMaxEll], sw[kMaxEll];
    const void* yhat[kMaxShift];
    double* z;
};

// calA runs on overlapping strips without halo loads (apply_calA_strip_body) on
// Dirichlet grids whose blocks fit one buffer range (N * 8 < 2^31 bytes); periodic
// grids and larger blocks use the halo-load form.  The tiling and the launch both
// follow this test.
inline bool calA_strips(const Geom& g) { return !g.periodic && g.n * 8 < (1ll << 31); }

struct CalAArgs {
    Geom g;
    Tiling t;
    const double* kappa;
    const double* x;
    const double* b;      // residual mode: y = b - calA x
    double* y;
    double* partial;      // residual mode: per-tile sum of squares
    int ell;
};

// Work list of a batched launch over independent problems: list entry q has
// arguments args[q] (the launch's own argument struct), owns blocks
// [first[q], first[q+1]) and belongs to problem pid[q]; live[pid] == 0 skips it and
// scale[pid] (forward transform only, may be null) multiplies its input.
struct BatchList {
    const void* args;
    const int* first;   // nprob + 1 entries
    const int* pid;
    const int* live;
    const double* scale;
    int nprob;
    int blocks;         // first[nprob]
    int wpb;            // waves per block, equal for every entry
};

enum BatchOp : int {
    BOP_FWD = 0,
    BOP_STEP = 1,
    BOP_FINAL = 2,
    BOP_CALA = 3,
    BOP_TRIPLE = 4,
    BOP_CALA_RES = 5,
    BOP_PAIR = 6
};

// Grid of the forward transform for n points: vx points per thread, 256 threads.
inline void fwd_geometry(long long n, int& vx, int& blocks) {
    vx = (n % 2 == 0) ? 2 : 1;
    const long long threads = (n + vx - 1) / vx;
    blocks = static_cast<int>((threads + 255) / 256);
}

// ---- launchers (stencil.hip) ----------------------------------------------
// prec: 0 = FP64 (double, kappa double), 1 = float + bf16 kappa, 2 = float + float kappa
// curk selects the stencil operand (SRC_RHAT: x_1 = rhat/theta, else a buffer);
// the kind of x_{k-1} travels in SweepArgs::prevk.
hipError_t launch_cheb_step(int ell, int prec, int curk, const void* args, hipStream_t s);
hipError_t launch_cheb_final(int ell, int prec, int curk, const void* args, hipStream_t s);
// Two steady steps per sweep (PairArgs<double> for prec 0, else PairArgs<float>).
hipError_t launch_cheb_pair(int prec, const void* args, hipStream_t s);
// Three steady steps per sweep (TripleArgs<double> for prec 0, else TripleArgs<float>).
hipError_t launch_cheb_triple(int prec, const void* args, hipStream_t s);
// Batched three-step sweeps (args TripleArgs per problem, L.wpb = their group count);
// code = 2 * first.
hipError_t launch_batch_triple(int prec, int code, int vx, const BatchList& L, hipStream_t s);
hipError_t launch_batch_pair(int prec, int vx, const BatchList& L, hipStream_t s);
hipError_t launch_tdft_fwd(int ell, int prec, const FwdArgs& a, hipStream_t s);
hipError_t launch_tdft_inv(int ell, int prec, const InvArgs& a, hipStream_t s);
hipError_t launch_apply_calA(int ell, bool resid, const CalAArgs& a, hipStream_t s);
// At most kAxpyFwdBlocks blocks (partial sums), nv <= 32.
constexpr int kAxpyFwdBlocks = 1024;
inline int axpy_fwd_blocks(long long n) {
    const int vx = (n % 2 == 0) ? 2 : 1;
    const long long blocks = ((n + vx - 1) / vx + 255) / 256;
    return static_cast<int>(blocks < kAxpyFwdBlocks ? blocks : kAxpyFwdBlocks);
}
hipError_t launch_axpy_fwd(int ell, int prec, const AxpyFwdArgs& a, hipStream_t s);
// Varying diagonal blocks: a.kappa holds l coefficient fields (block-major); residual
// mode writes l * tiles partials (index k * tiles + tile).
hipError_t launch_apply_calA_var(int ell, bool resid, const CalAArgs& a, hipStream_t s);
// One batched launch of op (BatchOp) for lists whose entries share l, precision,
// operand kind (sweeps), points per lane and waves per block; Dirichlet grids only.
hipError_t launch_batch(int op, int ell, int prec, int curk, int vx, const BatchList& L, hipStream_t s);

// ---- Krylov vector kernels (krylov.hip) ------------------------------------
struct VecSet {
    const double* v[kMaxBasis];
    double s2[kMaxBasis];  // squared scales of the raw basis vectors
};
int krylov_blocks();
// Partial sums go to partial[blk*nq_stride + q].
// mdot: q < nv: V_q . w, q = nv: w . w; with_last: q = nv+1+i (i < nv-1): V_i . V_{nv-1}
hipError_t launch_mdot(const VecSet& V, int nv, bool with_last, const double* w, long long len, double* partial,
                       int nq_stride, hipStream_t s);
// Same outputs for a basis with a fixed stride, vectors split over the waves of a block.
hipError_t launch_mdot_strided(const double* v0, long long vstride, int nv, bool with_last, const double* w,
                               long long len, double* partial, int nq_stride, hipStream_t s);
// axpy_norm: w -= sum_q c_q V_q with c_q = s2_q dcoef_q (dcoef on the device) or
// c_q = s2_q (dcoef == nullptr); q = 0: ||w||^2 after the update
hipError_t launch_axpy_norm(const VecSet& V, int nv, const double* dcoef, double* w, long long len, double* partial,
                            int nq_stride, hipStream_t s);
hipError_t launch_maxpy(const VecSet& Z, int nv, const double* coef_host_scaled, double* x, long long len,
                        hipStream_t s);
hipError_t launch_norm2(const double* w, long long len, double* partial, hipStream_t s);
// x = x + (d = a d + c z)
hipError_t launch_cheb_update(double* x, double* d, const double* z, double a, double c, long long len,
                              hipStream_t s);
hipError_t launch_reduce(const double* partial, int nblk, int nq, int nq_stride, double* out, hipStream_t s);

// ---- warm-start network (cnn.hip) ---------------------------------------------
// Parameters: [W1 (9x16x16), b1 (16), W2, b2, W3, b3], weights as [tap][out][in].
constexpr int kCnnParams = 3 * (9 * 256 + 16);

struct CnnConvArgs {
    const uint16_t* in;    // bf16 [B][H][W][16]
    const uint16_t* w;     // bf16 [9][16 out][16 in]
    const float* bias;     // [16] or null
    const uint16_t* mask;  // bf16 [B][H][W][16]: output zeroed where mask <= 0 (null: none)
    uint16_t* out16;       // bf16 [B][H][W][16] or null
    float* out32;          // float [B][H][W][nout] or null
    int nout;
    int B, H, W;
    int relu;
};

struct CnnWgradArgs {
    const uint16_t* act;  // layer input, bf16 [B][H][W][16]
    const uint16_t* dz;   // gradient of the layer output, bf16 [B][H][W][16]
    int B, H, W;
    float* partial;       // cnn_wgrad_waves(tiles) x (9*256 + 16)
};

struct CnnPrepArgs {
    Geom g;
    long long n;
    int ns;
    const void* rhat;                  // spectral buffer (inner real type)
    unsigned soff[kMaxShift];          // slot offsets (elements)
    int is_real[kMaxShift];
    float lam_re[kMaxShift], lam_im[kMaxShift];
    float inv_scale[kMaxShift], scale[kMaxShift];
    float fac_re[kMaxShift], fac_im[kMaxShift];  // complex factor applied to the output
    const double* kappa;
    double c0, c1;                     // input normalisation of ln kappa
    uint16_t* x;                       // bf16 [ns][N][16]
    float* rs;                         // optional: rhat / s per slot, float32 [ns][N][2] (re, im)
};

int cnn_wgrad_waves(long long ntiles);
hipError_t launch_cnn_conv(const CnnConvArgs& a, hipStream_t s);
hipError_t launch_cnn_wgrad(const CnnWgradArgs& a, float* grad, hipStream_t s);
hipError_t launch_cnn_loss(const float* y, const float* t, const float* tnorm, int B, int H, int W, int border,
                           uint16_t* dy16, float* partial, int* nblocks, hipStream_t s);
hipError_t launch_cnn_resloss(const float* y, const float* rhat, const float* kap, const float* lam,
                              const float* rnorm, int B, int H, int W, int border, float* e, uint16_t* dy16,
                              float* partial, int* nblocks, hipStream_t s);
hipError_t launch_cnn_adam(float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                           float bc1, float bc2, hipStream_t s);
hipError_t launch_cnn_weights(const float* w, uint16_t* wf, uint16_t* wb, float* bias, hipStream_t s);
hipError_t launch_cnn_prep(int prec, const CnnPrepArgs& a, hipStream_t s);
// all three layers per 16 x 16 tile in LDS, rhat and kappa read directly, x0 = scale * y
hipError_t launch_cnn_fused(int prec, const CnnPrepArgs& a, const uint16_t* wf, const float* bias, void* x0buf,
                            hipStream_t s);
hipError_t launch_cnn_post(int prec, const CnnPrepArgs& a, const float* y, void* x0buf, hipStream_t s);
hipError_t launch_cnn_resid(int prec, const CnnPrepArgs& a, const void* x0buf, const void* kap, double* partial,
                            int nblk, hipStream_t s);
hipError_t launch_zero_bytes(void* buf, long long off_bytes, long long nbytes, hipStream_t s);

// ---- exact shifted solves for a constant coefficient (exact.hip) -------------
// Slot s of a spectral buffer (interleaved complex, or real) maps to plane
// plane[s] (and plane[s] + 1 for the imaginary part) of a planar buffer of
// n-point planes; lambda_s = lr[s] + i li[s].
struct ExactArgs {
    long long n;
    int nx, ny, dim, nslot;
    double kappa;
    void* slot[kMaxShift];
    int cplx[kMaxShift];
    int plane[kMaxShift];
    double lr[kMaxShift], li[kMaxShift];
};
// prec 0: double, else float.  S: the even-mode and odd-mode halves of the n x n
// orthonormal DST-I matrix, column-major, ceil(n/2)^2 + floor(n/2)^2 entries.
long long dst_half_elems(int n);
hipError_t launch_dst_half(int prec, void* S, int n, hipStream_t s);
// split: spectral slots -> planes (with the even/odd butterfly along x); else the
// inverse butterfly from planes -> spectral slots
hipError_t launch_exact_planes(int prec, bool split, const ExactArgs& a, void* planes, hipStream_t s);
// In the sine basis along x, solve the tridiagonal systems along y of every slot:
// t holds the transformed right-hand sides (overwritten), the solutions go to u.
// carry: exact_carry_bytes(nx, ny, nslot) bytes of device scratch.
size_t exact_carry_bytes(int nx, int ny, int nslot);
hipError_t launch_exact_tridiag(int prec, const ExactArgs& a, void* t, void* u, void* carry, hipStream_t s);
// C = op(S) B for the half sine matrices (exact_gemm.hip): S d x d column-major
// (leading dimension d), B and C d x N with leading dimensions ldb, ldc; op(S) = S^T
// when trans; prec 0 float64, otherwise float32.
hipError_t launch_sine_gemm(int prec, bool trans, const void* S, int d, const void* B, int ldb, void* C, int ldc,
                            int N, hipStream_t s);

// ---- geometric multigrid for A - c I (mg.hip) --------------------------------
// Vertex-centred V-cycle: coarse point J = fine point 2J + 1 per coarsened dimension,
// harmonic face coarsening, linear interpolation, full weighting, two damped-Jacobi
// sweeps before and after, exact solve on the last level (at most 4 points).
constexpr int kMgMaxLevels = 32;
constexpr int kMgMaxVec = 2 * kMaxShift;
struct MgLevel {
    int nx, ny, dim;
    int cx, cy;  // made by coarsening x (y) of the previous level
    long long n;
    // wx / wy: face to the x+1 / y+1 neighbour (0 past the last point); bx0/bx1 (per
    // row) and by0/by1 (per column): Dirichlet faces; diag = 1 + all faces of a point
    double *diag, *wx, *wy, *bx0, *bx1, *by0, *by1;
    float *diag_f, *wx_f, *wy_f;  // float32 copies for the float32 cycle
};
struct MgHierarchy {
    int nlev;
    MgLevel lev[kMgMaxLevels];
};
// Level sizes of the hierarchy of a dim-dimensional nx x ny grid; returns the count.
int mg_plan(int dim, int nx, int ny, MgLevel* out);
// doubles of one level's arrays (the float32 copies included)
size_t mg_level_doubles(const MgLevel& L);
// Fills every level's arrays from the fine coefficient (pointers assigned by the caller).
hipError_t mg_build(const MgHierarchy& h, const double* kappa, hipStream_t s);
// scratch elements (of the vector type) of a V-cycle over nv vectors
size_t mg_scratch_elems(const MgHierarchy& h, int nv);
// u[v] = V-cycle applied to b[v] for the operator A - c[v] I (host arrays of nv <=
// kMgMaxVec device pointers / shifts); u may not alias b.  The float overload runs on
// the float32 copies of the level arrays (the coarsest solve stays float64).
hipError_t mg_vcycle(const MgHierarchy& h, int nv, const double* const* b, double* const* u, const double* c,
                     double* scratch, hipStream_t s);
hipError_t mg_vcycle(const MgHierarchy& h, int nv, const float* const* b, float* const* u, const double* c,
                     float* scratch, hipStream_t s);

// ---- saddle-point inner solves of P_SP (sp.hip) ---------------------------------
// nc complex shifts (MINRES on the real saddle form, P_D by V-cycles) and nr real
// shifts (CG, V-cycle preconditioner), iters iterations each, in lockstep.
struct SpProblem {
    const MgHierarchy* h;
    long long n;
    int nc, nr;
    double sigma[kMaxShift], rho[kMaxShift];  // complex: |Im lambda|, Re lambda
    int im_pos[kMaxShift];                    // complex: Im lambda > 0
    double lam[kMaxShift];                    // real shifts
    // slot data of the vector type (float64 or float32)
    const void* bc[kMaxShift];                // complex right-hand sides (interleaved, n points)
    void* yc[kMaxShift];                      // complex solutions (interleaved)
    const void* br[kMaxShift];                // real right-hand sides (n)
    void* yr[kMaxShift];                      // real solutions
};
// f32: float32 vectors and multigrid coefficients (inner products and scalars float64)
size_t sp_ws_bytes(const MgHierarchy& h, long long n, int nc, int nr, bool f32);
hipError_t sp_solve(const SpProblem& P, int iters, bool f32, void* ws, hipStream_t s);

// ---- batched FGMRES with device-resident scalars (batch_krylov.hip) -----------------
constexpr int kBKRed = 72;  // partial sums per block (2 * 32 dots + norm)
struct BKProb {
    const double* v0;   // basis V_i = v0 + i * vstride (i <= m)
    const double* z0;   // preconditioned vectors Z_i = z0 + i * vstride
    double* x;
    long long vstride, len;
    double* partial;    // nblk * kBKRed partial sums
    const double* partial2;  // per-tile partials of the residual form
    int ntiles;
    int nblk;           // blocks of the problem in a batched Krylov launch (<= 1024)
};
struct BKState {
    double H[(kMaxBasis) * (kMaxBasis - 1)];  // (m + 1) x m, row stride m
    double cs[kMaxBasis - 1], sn[kMaxBasis - 1], g[kMaxBasis], scale[kMaxBasis];
    double Lg[(kMaxBasis - 1) * (kMaxBasis - 1)], y[kMaxBasis - 1], coef[kMaxBasis];
    double bnorm, beta, orth;
    long long matvecs, ell, psum;
    int total, restarts, kdone, status, finished;
};
// blocks: the sum of the problems' nblk; live / cyc: per-problem masks
hipError_t launch_bk_mdot(const BKProb* P, int nprob, int blocks, const int* live, int nv, hipStream_t s);
hipError_t launch_bk_arnoldi(const BKProb* P, BKState* S, int nprob, const int* live, int j, int m, hipStream_t s);
hipError_t launch_bk_axpy_norm(const BKProb* P, const BKState* S, int nprob, int blocks, const int* live, int nv,
                               hipStream_t s);
hipError_t launch_bk_givens(const BKProb* P, BKState* S, int nprob, int* live, double* dscale, int j, int m,
                            double tol, int max_outer, hipStream_t s);
hipError_t launch_bk_update(const BKProb* P, BKState* S, int nprob, int blocks, const int* cyc, int m, hipStream_t s);
hipError_t launch_bk_cycle(const BKProb* P, BKState* S, int nprob, int* live, int* cyc, double* dscale, int m,
                           double tol, int max_outer, hipStream_t s);

// ---- setup kernels (setup.hip) -----------------------------------------------
hipError_t launch_kappa_setup(const Geom& g, const double* kappa, float* k32, uint16_t* k16, double* partial,
                              int nblk, hipStream_t s);
// Pointwise mean of l coefficient fields; bad[b] (setup_blocks() entries) counts the
// entries that are not finite and positive.
hipError_t launch_kappa_mean(const double* kb, int ell, long long n, double* mean, double* bad, hipStream_t s);
int setup_blocks();

// ---- host plumbing shared across translation units ---------------------------------
// Records msg as the calling thread's last error (ac_last_error) and returns status.
int set_error(int status, const std::string& msg);
// Device of a problem's context; a context's device and stream.
int problem_device(const ::ac_problem* p);
int ctx_device(const ::ac_ctx* c);
hipStream_t ctx_stream(const ::ac_ctx* c);
// Looks up, with that device current, the device address of the fixed scratch array of
// ac_apply_prec_noalloc for the device (once per device; noalloc.hip).
int noalloc_scratch_init(int device);

}  // namespace ac
