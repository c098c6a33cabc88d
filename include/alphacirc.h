/*
 * alphacirc: block alpha-circulant preconditioned all-at-once diffusion solves
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: Tabeart, Guerol, Pearson, Weaver, "Block alpha-circulant
 * preconditioners for all-at-once diffusion-based covariance operators".
 *
 *   All-at-once system (Section 1, eq. (1)):   calA x = b,
 *     calA = I_l (x) A - S (x) I_N, S the l x l down-shift, b = (b_1, 0, ..., 0).
 *   Preconditioner (eq. (2)):  P_alpha = I_l (x) A - C_alpha (x) I_N.
 *   Its inverse (eq. (4)):  scale by Gamma_alpha = diag(alpha^{(k-1)/l}),
 *     DFT across the l blocks, l shifted solves (A - lambda_j I) y_j = r_j
 *     (eq. (6)), inverse DFT, scale by Gamma_alpha^{-1}.
 *   Nested Chebyshev (Section 3): each shifted solve is p_j steps of Chebyshev
 *     semi-iteration on the segment S_j = [mu_lo - lambda_j, mu_hi - lambda_j]
 *     (Lemma 2, Proposition 1).
 *
 * Conventions for every entry point
 * ---------------------------------
 * Memory   All vector arguments are DEVICE pointers on the context's device,
 *          owned by the caller; the library never frees them.  Small arrays
 *          documented as "host" are host pointers.  The library allocates
 *          device memory only inside ac_ctx_create and ac_problem_create (and
 *          ac_cnn_create, ac_problem_create_multigrid) and frees it in the matching
 *          _destroy.
 * Layout   Block vectors are float64, block-major: x[k*N + i], k in [0, l),
 *          grid index i = iy*nx + ix (x fastest).  Cell-centred coefficient
 *          kappa[i] > 0, float64, length N.
 * Streams  All work is enqueued on the stream given to ac_ctx_create and is
 *          asynchronous with respect to the host, except where a function
 *          documents a synchronisation (ac_problem_create, ac_solve and the
 *          query functions).
 * Errors   Every function returns an ac_status; nothing throws across the ABI.
 *          A negative status is an error, with a message in ac_last_error()
 *          (per thread).  On error no output is guaranteed to be written.
 * Shifts   lambda_m = alpha^{1/l} exp(-2 pi i m / l), m = 0..l-1: the paper's
 *          shifts with the labelling conjugated so that they pair with the
 *          negative-exponent forward DFT (the pairing printed with eq. (3) does
 *          not diagonalise the down-shift C_alpha).  Because the block vectors are
 *          real, only the l_s = floor(l/2)+1 shifts m = 0..floor(l/2) are solved;
 *          the others are their complex conjugates.  Shift 0 and (l even) shift
 *          l/2 are real.
 */
#ifndef ALPHACIRC_H
#define ALPHACIRC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ac_ctx ac_ctx;         /* device, stream, pinned staging, kernel timers */
typedef struct ac_problem ac_problem; /* one grid + kappa field, one l, one alpha */

typedef enum {
    AC_OK = 0,
    AC_NOT_CONVERGED = 1,    /* non-fatal: ac_solve hit max_outer; info is filled in */
    AC_ERR_ARG = -1,         /* invalid argument (null pointer, size, option) */
    AC_ERR_ALPHA = -2,       /* alpha outside (0, mu_lo^l) (Corollary 1, Lemma 1) */
    AC_ERR_BOUNDS = -3,      /* spectral bounds not 1 <= mu_lo <= mu_hi, finite */
    AC_ERR_HIP = -4,         /* a HIP runtime call failed */
    AC_ERR_WORKSPACE = -5,   /* workspace pointer null or smaller than required */
    AC_ERR_NONFINITE = -6,   /* kappa not finite and positive, or a solve produced NaN/Inf */
    AC_ERR_UNSUPPORTED = -7  /* e.g. l outside [2, 16], l*N >= 2^31, restart_m > 32 */
} ac_status;

typedef enum { AC_BC_DIRICHLET = 0, AC_BC_PERIODIC = 1 } ac_bc;

/* Arithmetic of the inner (time-DFT + shifted Chebyshev) part.  The outer
 * operator, Krylov basis, residuals and solution are always float64.
 *   AC_PREC_FP64        complex128 iterates, float64 kappa
 *   AC_PREC_MIXED_BF16K complex64 iterates, bfloat16 kappa (round to nearest even)
 *   AC_PREC_MIXED_FP32K complex64 iterates, float32 kappa */
typedef enum { AC_PREC_FP64 = 0, AC_PREC_MIXED_BF16K = 1, AC_PREC_MIXED_FP32K = 2 } ac_precision;

/* Inner shifted solves.  Chebyshev from a zero initial guess (the paper's method), or
 * from the learned warm start attached with ac_problem_attach_cnn (makes the
 * preconditioner nonlinear): for every preconditioner application
 * (AC_INNER_CHEB_CNN), or only for the first vector of each FGMRES cycle, the true
 * residual, with zero guesses inside the cycle (AC_INNER_CHEB_CNN_CYCLE), or as a
 * minimal-residual correction before each FGMRES cycle: z = the warm-started P^{-1}
 * of the true residual r, x += gamma z with gamma = <calA z, r> / |calA z|^2 (the
 * residual cannot grow), then a plain cycle (AC_INNER_CHEB_CNN_MR; one extra
 * preconditioner application and calA product per cycle).  ac_apply_prec treats both
 * cycle modes as AC_INNER_CHEB_CNN.
 * AC_INNER_EXACT applies P_alpha^{-1} itself (eq. (4) with direct shifted solves; the
 * paper's reference preconditioner, Section 2 and Fig. 2): only for a constant
 * coefficient on a Dirichlet grid, where the sine transform of Appendix A diagonalises
 * A along x and every shifted solve reduces to tridiagonal systems along y (dense
 * transforms by the library's matrix-core products in the inner precision).  p_uniform
 * and p_per_shift are
 * ignored and count no products with A.  AC_ERR_UNSUPPORTED for a varying coefficient
 * (or varying diagonal blocks whose mean is not constant) or periodic grids.
 * AC_INNER_SP is the saddle-point preconditioner P_SP (Section 4): each complex shift's
 * system in the real saddle form of eq. (saddlesystem), solved by preconditioned MINRES
 * with P_D of eq. (minresprecond), each real shift by preconditioned CG (Section 5),
 * P_D and the CG preconditioner applied by one geometric multigrid V-cycle (built by
 * ac_problem_create_multigrid; the paper uses a black-box algebraic multigrid there).
 * p_uniform (or equal p_per_shift entries) iterations per shift from a zero guess;
 * float64 (AC_PREC_FP64) or float32 vectors and multigrid coefficients with float64
 * inner products and recurrence scalars (AC_PREC_MIXED_FP32K; bf16 is refused); nonlinear (use FGMRES, or the outer Chebyshev iteration as the paper
 * does); two products with A per MINRES step and one per CG step are counted. */
typedef enum {
    AC_INNER_CHEB = 0,
    AC_INNER_CHEB_CNN = 1,
    AC_INNER_CHEB_CNN_CYCLE = 2,
    AC_INNER_EXACT = 3,
    AC_INNER_SP = 4,
    AC_INNER_CHEB_CNN_MR = 5
} ac_inner;

typedef struct {
    int dim;   /* 1 or 2 */
    int nx;    /* >= 1 */
    int ny;    /* >= 1; must be 1 when dim == 1 */
    int bc;    /* ac_bc */
} ac_grid;

typedef struct {
    double mu_lo;  /* lower end of an interval enclosing the spectrum of A */
    double mu_hi;  /* upper end */
} ac_bounds;

/* Outer iteration of ac_solve:
 *   AC_OUTER_FGMRES     right-preconditioned flexible GMRES(restart_m);
 *   AC_OUTER_CHEBYSHEV  the paper's outer solver: Chebyshev semi-iteration on
 *                       P^{-1} calA with the eigenvalue interval of Corollary 1,
 *                       [1, mu_lo^l / (mu_lo^l - alpha)], mu_lo the lower spectral bound
 *                       of A; valid for a linear preconditioner (AC_INNER_CHEB,
 *                       AC_INNER_EXACT); also run with AC_INNER_SP, whose inner
 *                       MINRES / CG make it nonlinear (the paper's setting).  Not with
 *                       AC_PREC_MIXED_BF16K (AC_ERR_UNSUPPORTED): bf16 rounding of kappa
 *                       moves the eigenvalues of P^{-1} calA out of that interval, whose
 *                       width is about alpha / mu_lo^l. */
typedef enum { AC_OUTER_FGMRES = 0, AC_OUTER_CHEBYSHEV = 1 } ac_outer;

typedef struct {
    int precision;           /* ac_precision */
    int inner;               /* ac_inner */
    const int* p_per_shift;  /* host, l entries (entry m pairs with lambda_m; conjugate
                                entries must be equal), or NULL to use p_uniform */
    int p_uniform;           /* inner Chebyshev steps per shift when p_per_shift == NULL */
    double tol;              /* ac_solve: stop when ||b - calA x||_2 / ||b||_2 <= tol */
    int restart_m;           /* ac_solve: FGMRES restart length, 1..32 (also >= 1 for Chebyshev) */
    int max_outer;           /* ac_solve: maximum total outer iterations */
    int outer;               /* ac_outer (0 = FGMRES) */
} ac_solve_opts;

typedef struct {
    int outer_iters;          /* FGMRES iterations (preconditioner applications) */
    int restarts;             /* completed FGMRES cycles */
    long long matvecs_A;      /* products with A, counted as in Table 1: l per calA,
                                 p_j per shift per preconditioner application (all l shifts) */
    double rel_residual_true; /* ||b - calA x|| / ||b|| of the returned x, float64 */
    double seconds;           /* wall time of the solve (host clock, includes syncs) */
    int cnn_fallbacks;        /* shifted solves where the warm start was rejected */
    int reserved;
    double orth_loss;         /* max |q_i . q_k|, i != k, over the Krylov bases built */
} ac_solve_info;

/* Kernel classes timed when profiling is on (ac_ctx_set_profiling). */
typedef enum {
    AC_K_TDFT_FWD = 0,   /* forward scaled time-DFT (+ conversion to the inner type) */
    AC_K_CHEB_STEP = 1,  /* one steady-state batched shifted Chebyshev sweep, all active shifts */
    AC_K_CHEB_FINAL = 2, /* last Chebyshev sweep fused with the inverse scaled time-DFT */
    AC_K_APPLY_CALA = 3, /* calA x or b - calA x, float64 */
    AC_K_KRYLOV = 4,     /* multi-dot / multi-axpy / norms, float64 */
    AC_K_CNN = 5,        /* warm-start network */
    AC_K_CHEB_FIRST = 6, /* the first sweep from a zero guess (x_2 from x_1 = rhat/theta) */
    AC_K_EXACT = 7,      /* AC_INNER_EXACT: sine transforms, tridiagonal solves, inverse time-DFT */
    AC_K_SADDLE = 8,     /* AC_INNER_SP: MINRES / CG with multigrid V-cycles (whole inner solve) */
    AC_K_CHEB_PAIR = 9,  /* two steady Chebyshev sweeps fused into one (per shift group) */
    AC_K_CHEB_TRIPLE = 10, /* three steady Chebyshev sweeps fused into one (per shift group) */
    AC_K_COUNT = 11
} ac_kernel_class;

/* ---- status ------------------------------------------------------------- */
const char* ac_status_string(int status);
/* Detail of the last error on the calling thread ("" if none). */
const char* ac_last_error(void);

/* ---- context ------------------------------------------------------------ */
/* Binds a device and a stream.  hip_stream is a hipStream_t (NULL = default
 * stream); the caller keeps it alive until ac_ctx_destroy. */
int ac_ctx_create(int device, void* hip_stream, ac_ctx** out);
int ac_ctx_destroy(ac_ctx* ctx);
int ac_ctx_set_stream(ac_ctx* ctx, void* hip_stream);
/* Graph replay of launch-bound inner solves (default on): the AC_INNER_SP inner solve
 * (hundreds of small launches per application) is captured once per problem, workspace,
 * step count and precision on a stream the context owns and replayed as one hipGraph on
 * the context stream; off runs the same kernels directly.  Results are identical. */
int ac_ctx_set_graphs(ac_ctx* ctx, int on);
/* Profiling: when on, every launch of the classes above is bracketed by HIP events
 * on the context stream and its algorithmic bytes are accumulated. */
int ac_ctx_set_profiling(ac_ctx* ctx, int on);
/* Synchronises the stream, then returns per class the summed kernel milliseconds,
 * launch count and algorithmic bytes since the last reset (host arrays of
 * AC_K_COUNT entries; any may be NULL). */
int ac_ctx_kernel_stats(ac_ctx* ctx, double* ms, long long* launches, double* bytes);
int ac_ctx_reset_stats(ac_ctx* ctx);
/* Marching-stencil tile shape for the Chebyshev sweeps (0 = automatic):
 * rows_per_wave in [0, 4096], waves_per_block in [0, 4], points_per_lane in [0, 2]
 * (2 needs an even nx >= 128; otherwise 1 is used).  Results do not depend on it. */
int ac_ctx_set_tiling(ac_ctx* ctx, int rows_per_wave, int waves_per_block, int points_per_lane);

/* ---- problem ------------------------------------------------------------ */
/* Builds A from the grid and the cell-centred kappa (device, N float64, read
 * during the call; a float64 copy and the float32/bfloat16 copies are kept):
 *   (A u)_i = u_i + sum over faces f of kappa_f (u_i - u_nb),
 *   kappa_f = (kappa_i + kappa_nb)/2; a Dirichlet boundary face uses kappa_i and
 *   a zero ghost value; periodic faces wrap.  Constant kappa gives I + kappa (-Delta_h),
 *   the paper's operator (Section 5, eq. (IminusLap)) with kappa = nu/h^2.
 * bounds == NULL: computes an enclosing interval on the device: mu_hi = the
 * Gershgorin maximum over rows, mu_lo = 1 + min(kappa) * lambda_min(-Delta_h)
 * (lambda_min of the integer Dirichlet stencil; 0 for periodic).  The interval
 * feeds the Chebyshev centres (Proposition 1).  Checks 0 < alpha < mu_lo^l
 * (Corollary 1) and l in [2, 16].  AC_ERR_UNSUPPORTED when l*N (plus 64 values of
 * padding per frequency) reaches 2^31: block vectors are addressed with 32-bit
 * element offsets.  Synchronises the stream. */
int ac_problem_create(ac_ctx* ctx, const ac_grid* grid, const double* kappa_dev, int ell, double alpha,
                      const ac_bounds* bounds, ac_problem** out);
int ac_problem_destroy(ac_problem* p);

/* Multigrid hierarchy of A for AC_INNER_SP (no paper definition: the paper uses a
 * black-box AMG).  Vertex-centred geometric V-cycle: each dimension of n > 1 points
 * coarsens to floor(n/2) (coarse point J = fine point 2J + 1) until at most 4 points
 * remain; coarse face coefficients are the harmonic combination of the two fine faces
 * in series divided by 4 (a Dirichlet face at the high end of an even n: halved),
 * averaged 1/4, 1/2, 1/4 along a coarsened tangential direction; linear interpolation,
 * full weighting, two damped-Jacobi sweeps (omega 0.8) before and after, an exact
 * solve on the last level.  Built from the problem's float64 coefficient (for varying
 * blocks: their mean, the representative block), owned by the problem, freed by
 * ac_problem_destroy; a second call does nothing.  Dirichlet grids only.
 * Synchronises. */
int ac_problem_create_multigrid(ac_problem* p);
/* Device bytes for ac_mg_vcycle over nvec vectors (1 <= nvec <= 18). */
int ac_mg_workspace_size(const ac_problem* p, int nvec, size_t* bytes);
/* u_q = one V-cycle for (A - shifts[q] I) u_q = b_q from zero, q < nvec: b and u hold
 * nvec vectors of N float64 back to back (u may not alias b); shifts is a host array,
 * each shift below mu_lo (so that A - c I is SPD). */
int ac_mg_vcycle(ac_problem* p, int nvec, const double* shifts, const double* b, double* u, void* ws,
                 size_t ws_bytes);
/* Varying diagonal blocks A_1, ..., A_l (the extension named in the Conclusions):
 * calA = blockdiag(A_k) - S (x) I_N with A_k built from the k-th coefficient field of
 * kappa_blocks (device, l * N float64, block-major, each finite and positive).  The
 * preconditioner uses the representative block A(mean_k kappa_k), which equals the
 * mean of the A_k (A is affine in kappa); its spectral bounds and the alpha check
 * refer to that block.  Every ac_* call on the problem then applies the varying
 * blocks in calA (ac_apply_A, the residuals of ac_solve).  Corollary 1 no longer
 * bounds the spectrum, so the outer Chebyshev iteration and batched solves return
 * AC_ERR_UNSUPPORTED; FGMRES is the outer solver.  The l*N limit of ac_problem_create
 * applies.  Synchronises. */
int ac_problem_create_blocks(ac_ctx* ctx, const ac_grid* grid, const double* kappa_blocks, int ell, double alpha,
                             const ac_bounds* bounds, ac_problem** out);
/* Interval used for the FP64 inner solve (host outputs). */
int ac_spectral_bounds(const ac_problem* p, double* mu_lo, double* mu_hi);
/* Sizes: N, l and l_s = floor(l/2) + 1 (host outputs, any may be NULL). */
int ac_problem_dims(const ac_problem* p, long long* n, int* ell, int* n_shifts);
/* The shifts of eq. (3) with the sign of the forward transform used here:
 * lambda_m = alpha^{1/l} exp(-2 pi i m / l), m = 0..l-1; lam: host, 2 l doubles
 * (Re, Im pairs). */
int ac_problem_shifts(const ac_problem* p, double* lam);

/* ---- inner-iteration allocation (Section 5.1, Table 1) ------------------- */
/* NC2, Algorithm 1: sigma_m from the condition number of Re(A - lambda_m I),
 * r_m = ln(sigma_0)/ln(sigma_m), normalised, p_m = floor(r_m * budget), clamped
 * to >= 1 (a zero would drop a frequency).  budget is the total inner budget
 * (the paper's l * n_x * eta).  p_out: host, l entries. */
int ac_alloc_nc2(const ac_problem* p, double budget, int* p_out);
/* NC1: floor(budget / l) for every shift, clamped to >= 1. */
int ac_alloc_nc1(const ac_problem* p, double budget, int* p_out);

/* ---- workspaces ----------------------------------------------------------- */
/* Device bytes needed by ac_apply_prec / ac_shifted_cheb (prec) and ac_solve. */
int ac_prec_workspace_size(const ac_problem* p, const ac_solve_opts* opts, size_t* bytes);
int ac_solve_workspace_size(const ac_problem* p, const ac_solve_opts* opts, size_t* bytes);

/* ---- operators (Section 1 eq. (1); Section 2.2 eq. (4); Section 3) ------- */
/* y = calA x: y_k = A x_k - x_{k-1}, x_0 := 0 (float64; x, y: l*N, must not overlap:
 * AC_ERR_ARG). */
int ac_apply_A(ac_problem* p, const double* x, double* y);

/* z = P_NC^{-1} r (nested Chebyshev, opts->precision / p_per_shift / inner), the
 * three steps fused into first/last Chebyshev sweeps.  With p_m -> infinity this
 * tends to the exact P_alpha^{-1} r of eq. (4).  r, z: l*N float64, must not overlap
 * (AC_ERR_ARG). */
int ac_apply_prec(ac_problem* p, const ac_solve_opts* opts, const double* r, double* z, void* ws, size_t ws_bytes);

/* z = P_NC^{-1} r exactly as ac_apply_prec (AC_INNER_CHEB only), for callers that
 * cannot allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): no workspace argument, no allocation.  The
 * workspace is a fixed array of AC_NOALLOC_SCRATCH_BYTES in device memory that every
 * GPU the library runs on holds until the process ends (its address is looked up once
 * per device by ac_ctx_create).  Problems whose ac_prec_workspace_size exceeds it
 * return AC_ERR_WORKSPACE (e.g. 512 x 512 with l = 10 fits in complex64, not in
 * float64); other inner modes AC_ERR_UNSUPPORTED.  All calls on one device share the
 * array: calls that overlap in time on one device (several host threads or streams)
 * race; serialise them.  r, z: l*N float64, must not overlap (AC_ERR_ARG).
 * Asynchronous on the context's stream; with profiling off it calls no allocating
 * runtime or library routine. */
#define AC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ac_apply_prec_noalloc(ac_problem* p, const ac_solve_opts* opts, const double* r, double* z);

/* Spectral buffers used by the three stages below: l_s shift slices, slice m of
 * ac_spectral_offsets()[m] elements of the inner real type (float64 for
 * AC_PREC_FP64, float32 otherwise), real shifts (m = 0, and m = l/2 for even l) as
 * N reals, complex shifts as N interleaved (re, im) pairs.  offsets: host array of
 * l_s + 1 entries (last = total elements). */
int ac_spectral_offsets(const ac_problem* p, int precision, long long* offsets);
/* rhat_m = sum_k alpha^{k/l} r_k exp(-2 pi i m k / l), m = 0..l_s-1 (unnormalised). */
int ac_tdft_forward(ac_problem* p, int precision, const double* r, void* rhat);
/* yhat_m = p_m Chebyshev steps on (A - lambda_m I) y = rhat_m from zero (or from x0hat
 * when non-NULL, same layout).  yhat may not alias rhat.  AC_ERR_UNSUPPORTED for
 * inner = AC_INNER_EXACT. */
int ac_shifted_cheb(ac_problem* p, const ac_solve_opts* opts, const void* rhat, const void* x0hat, void* yhat,
                    void* ws, size_t ws_bytes);
/* z_k = alpha^{-k/l} (1/l) Re sum_{m=0}^{l-1} yhat_m exp(+2 pi i m k / l), using
 * yhat_{l-m} = conj(yhat_m). */
int ac_tdft_inverse(ac_problem* p, int precision, const void* yhat, double* z);

/* rel[m] = ||rhat_m - (A - lambda_m I) yhat_m|| / ||rhat_m||, m = 0..l_s-1 (host output),
 * the inner residual of shifted solutions in the spectral layout (float64 sums).
 * Meant for judging warm-start guesses: lambda is taken in float32 and the norm is
 * formed from |rhat|^2, <B yhat, rhat> and |B yhat|^2, so values below about 1e-7 are
 * not resolved.  Synchronises. */
int ac_shifted_residual(ac_problem* p, int precision, const void* rhat, const void* yhat, double* rel);

/* ---- outer solve ---------------------------------------------------------- */
/* Right-preconditioned flexible GMRES(restart_m) on calA x = b with P_NC^{-1},
 * Arnoldi by modified Gram-Schmidt in inverse compact WY form (two sweeps over
 * the basis per step), all in float64; Givens
 * rotations on the host.  x holds the initial guess on entry and the solution on
 * return; b and x must not overlap (AC_ERR_ARG).  Converged when the TRUE relative residual ||b - calA x||/||b|| <= tol
 * (the paper's residual definition, Section 5).  A zero b gives x = 0 and zeroed
 * info, with no iteration.  Synchronises once per iteration.  info may be NULL.
 * Returns AC_NOT_CONVERGED after max_outer. */
int ac_solve(ac_problem* p, const ac_solve_opts* opts, const double* b, double* x, void* ws, size_t ws_bytes,
             ac_solve_info* info);
/* ac_solve that also copies the first rec_count vectors handed to the
 * preconditioner (the Arnoldi basis vectors v_j, unnormalised, in order; device,
 * rec_count * l * N float64) into rec; *recorded (host) receives how many were
 * written.  Used to draw training inputs for the warm start from the plain method.
 * Synchronises. */
int ac_solve_record(ac_problem* p, const ac_solve_opts* opts, const double* b, double* x, void* ws,
                    size_t ws_bytes, ac_solve_info* info, double* rec, int rec_count, int* recorded);

/* Steady Chebyshev sweeps in shift groups: mode -1 (default) groups problems with 5
 * or more unique shifts, 0 never, 1 always.  A group holds at most one real and two
 * complex shifts and runs as its own launch; results are those of the all-shift
 * sweep.  Problems with grouped sweeps default to 8 rows per wave. */
int ac_ctx_set_shift_groups(ac_ctx* ctx, int mode);

/* Two steady Chebyshev steps per sweep (temporal blocking of the three-term recurrence
 * of Section 3): mode 1 (default) fuses every two consecutive steady steps in which the
 * same shifts compute, on Dirichlet grids, into one sweep per shift group (one real,
 * two complex shifts) that reads x_k, x_{k-1} and rhat once and writes x_{k+1} and
 * x_{k+2}; mode 0 runs single steps.  The iterates are those of single steps up to
 * rounding (operations may be contracted differently: a few ulps per step).  rows_per_wave, waves_per_block (1..4) and
 * points_per_lane (1..2) set the paired sweep's tiling, 0 = automatic (rows for about
 * one round of waves, 4..32; 4 waves; 2 points per lane in float32 on even grids at
 * least 128 wide, else 1).  Pairs
 * are used while every spectral buffer is below 2^31 bytes.  Profiling (AC_K_CHEB_PAIR)
 * counts the two steps' unfused algorithmic bytes.
 * Batched solves (ac_batch_solve) run single steps. */
int ac_ctx_set_step_pairs(ac_ctx* ctx, int mode, int rows_per_wave, int waves_per_block, int points_per_lane);

/* Three steady Chebyshev steps per sweep (Section 3's recurrence, temporally blocked):
 * mode 1 (default) fuses runs of steady steps in which the same shifts compute into
 * blocks of three (a remainder of two as a pair, of one as a single step), where pairs
 * are allowed (mode 1 of ac_ctx_set_step_pairs, Dirichlet grids, buffers below 2^31
 * bytes); the first three steps from a zero guess form a block too.  A block reads
 * x_k, x_{k-1} and rhat once and writes x_{k+2} and x_{k+3} (x_{k+1} stays in
 * registers), in one launch over every shift: a workgroup per tile (a strip of grid
 * columns by rows_per_wave rows) with one wave per shift group (the real shifts
 * together, each complex shift alone).  The iterates are those of single steps up to
 * rounding (a few ulps per step).  rows_per_wave 0 picks the height for about one round
 * of workgroups at waves_per_simd waves per SIMD (0: 4); points_per_lane 0 picks 2 in
 * float32 on even grids at least 128 wide, else 1.  Profiling (AC_K_CHEB_TRIPLE,
 * AC_K_CHEB_FIRST) counts each launch's own minimum bytes: the vector streams it
 * reads and writes once each and kappa once. */
int ac_ctx_set_step_triples(ac_ctx* ctx, int mode, int rows_per_wave, int waves_per_simd, int points_per_lane);

/* ---- measurement ------------------------------------------------------------
 * Streaming-bandwidth calibration (not part of the method): times reps passes of one
 * kernel that reads `reads` and writes `writes` contiguous streams (each 0..4, not both
 * zero) of equal length carved from ws (16-byte aligned; ws_bytes / (16 (reads +
 * writes)) float32x4 elements per stream, at least 1024), plain loads and non-temporal
 * stores, on the context's stream.  gbps (host): bytes moved per second / 1e9, the
 * ceiling for a memory-bound kernel with that read / write mix.  Overwrites ws (zeroes it
 * first).  Synchronises. */
int ac_stream_bandwidth(ac_ctx* ctx, int reads, int writes, void* ws, size_t ws_bytes, int reps, double* gbps);

/* ---- tiling ----------------------------------------------------------------
 * Sweep tiling of one problem (overrides the context's ac_ctx_set_tiling; 0 keeps
 * the context's value): rows per wave, waves per block (1..4), points per lane
 * (1 or 2; 1 is forced for odd or narrow grids).  It applies to single sweeps (the
 * first and last ones, and steady steps not fused); fused blocks of steady steps take
 * the tiling of ac_ctx_set_step_pairs / ac_ctx_set_step_triples. */
int ac_problem_set_tiling(ac_problem* p, int rows_per_wave, int waves_per_block, int points_per_lane);
/* Tile tuner: times the shifted Chebyshev sweeps of p at the given precision for
 * candidate tilings (points per lane 1 and 2, 4..64 rows per wave, 1, 2 or 4 waves
 * per block), keeps the fastest for p (single and batched solves), and, when
 * cache_path is not NULL, records it in that JSON file keyed by (nx, ny, l,
 * precision); an entry already there is applied without timing.  ws: a device
 * workspace of ac_prec_workspace_size bytes for the plain inner solver (its contents
 * are overwritten).  out (host, 3 ints, may be NULL): rows per wave, waves per block,
 * points per lane; us (may be NULL): time per sweep in microseconds (0 when taken
 * from the cache).  Synchronises. */
int ac_tune_tiling(ac_problem* p, int precision, const char* cache_path, void* ws, size_t ws_bytes, int* out,
                   double* us);

/* ---- batched solves ------------------------------------------------------
 * Solves count independent systems calA_q x_q = b_q (eq. (1)), each with its own
 * grid, coefficient field, l and alpha, as ac_solve does one: the FGMRES iterations
 * of all problems advance in lockstep, every stencil stage runs as one launch per
 * kernel variant over a work list of all problems' tiles, the per-iteration launch
 * sequence is captured once into a hipGraph per Arnoldi index and replayed, and a
 * problem that has converged is masked out of every later launch.  Sweep tiles
 * follow each problem's tiling (ac_tune_tiling).
 * Requirements: every problem on ctx, Dirichlet grids, opts shared by all with
 * inner = AC_INNER_CHEB and p_per_shift = NULL (uniform p_uniform); count <= 256.
 * b, x: host arrays of count device pointers (x: initial guess in, solution out).
 * infos: host array of count entries or NULL.  Runs on a stream of its own after
 * synchronising the context stream (kernel profiling is suspended); synchronises
 * before returning.  Returns AC_NOT_CONVERGED if any problem reached max_outer. */
int ac_batch_workspace_size(ac_ctx* ctx, int count, ac_problem* const* problems, const ac_solve_opts* opts,
                            size_t* bytes);
int ac_batch_solve(ac_ctx* ctx, int count, ac_problem* const* problems, const ac_solve_opts* opts,
                   const double* const* b, double* const* x, void* ws, size_t ws_bytes, ac_solve_info* infos);

/* ---- learned warm start (not part of the paper's method) ----------------------
 * A three-layer 3x3 convolutional network (5 -> 16 -> 16 -> 2 channels, ReLU after
 * the first two layers, zero padding), bfloat16 weights/activations with float32
 * accumulation on the matrix cores, gives the initial guess of each shifted inner
 * solve; the Chebyshev steps then correct it (AC_INNER_CHEB_CNN).  Inputs per shift
 * m and grid point: Re rhat_m / s_m, Im rhat_m / s_m, Re lambda_m, Im lambda_m,
 * (ln kappa - c0) / c1 with s_m = RMS(rhat_m); outputs Re x0_m / s_m, Im x0_m / s_m.
 * Each guess is multiplied by the complex factor c_m that minimises
 * ||rhat_m - c_m (A - lambda_m) x0_m|| (a one-dimensional minimal-residual step; can be
 * switched off), and a guess with ||rhat_m - (A - lambda_m) x0_m|| >= tau ||rhat_m||
 * (tau = 1 by default), or not finite, is replaced by zero (counted in
 * ac_solve_info.cnn_fallbacks); see ac_cnn_set_guess_policy.
 * Parameter vector (float, host): [W1, b1, W2, b2, W3, b3], each W as [tap = 3 ky + kx]
 * [out 16][in 16] and each b as [16]; entries beyond 5 inputs (layer 1) and 2 outputs
 * (layer 3) are held at zero.
 * Tensors are NHWC with 16 channels: x bf16 bits [B][H][W][16] (uint16), targets and
 * outputs float [B][H][W][2]. */
typedef struct ac_cnn ac_cnn;
int ac_cnn_param_count(void);
int ac_cnn_create(ac_ctx* ctx, ac_cnn** out);          /* all parameters zero */
int ac_cnn_destroy(ac_cnn* cnn);
/* Copies parameters (host, ac_cnn_param_count() floats) and the ln kappa normalisation;
 * resets the optimiser state.  Synchronises. */
int ac_cnn_set_params(ac_cnn* cnn, const float* params, double c0, double c1);
int ac_cnn_get_params(const ac_cnn* cnn, float* params, double* c0, double* c1);
/* Device workspace for ac_cnn_forward / ac_cnn_grad on a batch of B images H x W. */
int ac_cnn_workspace_size(int batch, int height, int width, size_t* bytes);
int ac_cnn_forward(ac_cnn* cnn, const uint16_t* x, int batch, int height, int width, float* y, void* ws,
                   size_t ws_bytes);
/* Loss L = (1/B) sum_b sum_mask |y_b - t_b|^2 / tnorm_b (mask: cells at least `border`
 * away from the image edge; tnorm_b = sum_mask |t_b|^2, device floats) and its gradient
 * with respect to every parameter (kept for ac_cnn_adam_step; copied to grad if not
 * NULL).  Synchronises. */
int ac_cnn_grad(ac_cnn* cnn, const uint16_t* x, const float* t, const float* tnorm, int border, int batch,
                int height, int width, void* ws, size_t ws_bytes, double* loss, float* grad);
/* Residual-space loss of the shifted solves of Section 3 on crops:
 * L = (1/B) sum_b sum_mask |rhat_b - (A_b - lambda_b) y_b|^2 / rnorm_b, y_b the network
 * output read as a complex field, A_b the five-point operator of the coefficient crop
 * kappa_b (face value (kappa_i + kappa_nb)/2), rnorm_b = sum_mask |rhat_b|^2.  Device
 * arrays: rhat float [B][H][W][2] (the same scaled field as input channels 0, 1),
 * kappa float [B][H][W], lam float [B][2] (Re, Im of the crop's shift), rnorm float
 * [B].  border >= 1 (every masked point's neighbours lie in the crop), else
 * AC_ERR_ARG.  Same workspace, gradient and synchronisation as ac_cnn_grad. */
int ac_cnn_grad_residual(ac_cnn* cnn, const uint16_t* x, const float* rhat, const float* kappa, const float* lam,
                         const float* rnorm, int border, int batch, int height, int width, void* ws,
                         size_t ws_bytes, double* loss, float* grad);
/* One Adam step (bias-corrected) with the last gradient. */
int ac_cnn_adam_step(ac_cnn* cnn, double lr, double beta1, double beta2, double eps);
/* Network inputs x (device bf16 [l_s][N][16]) for every shift slot of a spectral
 * buffer rhat (layout of ac_spectral_offsets): channels Re rhat_m / s_m, Im rhat_m / s_m,
 * Re lambda_m, Im lambda_m, (ln kappa - c0) / c1, the rest zero, s_m the RMS of rhat_m;
 * slot order m = 0, then m = l/2 (even l), then m = 1, 2, ...; scales: host, l_s RMS
 * values in slot order (or NULL); rscaled: device float32 [l_s][N][2], (Re, Im) of
 * rhat_m / s_m in float32 (the training target's right-hand side), or NULL. */
int ac_cnn_make_inputs(ac_problem* p, const ac_cnn* cnn, int precision, const void* rhat, uint16_t* x,
                       double* scales, float* rscaled);
/* The attached network's initial guesses x0hat (spectral layout) for every shift of
 * rhat, exactly as AC_INNER_CHEB_CNN forms them (scaling and fallback included);
 * rejected (host, may be NULL) receives the number of slots reset to zero.  Workspace
 * from ac_cnn_guess_workspace_size.  Synchronises. */
int ac_cnn_guess_workspace_size(const ac_problem* p, size_t* bytes);
int ac_cnn_guess(ac_problem* p, int precision, const void* rhat, void* x0hat, void* ws, size_t ws_bytes,
                 int* rejected);
/* Inference kernels for the guesses: fused != 0 (default) evaluates all three layers
 * per 16 x 16 tile in LDS straight from rhat and kappa; 0 runs input packing, three
 * convolution launches and output scaling (the training kernels).  Same results. */
int ac_cnn_set_inference(ac_cnn* cnn, int fused);
/* Guess policy: scaling != 0 (default) multiplies each guess by its
 * residual-minimising complex factor; a guess is kept only if
 * ||rhat_m - (A - lambda_m) x0_m|| < accept_ratio ||rhat_m||, accept_ratio in (0, 1]
 * (default 1, the plain fallback rule). */
int ac_cnn_set_guess_policy(ac_cnn* cnn, int scaling, double accept_ratio);
/* Attaches the network used by AC_INNER_CHEB_CNN (NULL detaches; not owned). */
int ac_problem_attach_cnn(ac_problem* p, ac_cnn* cnn);

#ifdef __cplusplus
}
#endif
#endif /* ALPHACIRC_H */
