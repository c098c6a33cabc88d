// C ABI of alphacirc: the outer solves (flexible GMRES with one-reduction modified
// Gram-Schmidt, or the outer Chebyshev iteration) around the preconditioner of api.hip.
#include "host.h"

using namespace ach;

// ---------------------------------------------------------------------------
// FGMRES

namespace {
// Products with A per preconditioner application, counted over all l shifts as in
// Table 1: p_m per Chebyshev solve; for P_SP two per MINRES step (complex shifts) and
// one per CG step (real shifts); none for the exact solve.
long long prec_products(const ac_problem* p, const ac_solve_opts* o, const std::vector<int>& pm) {
    if (o->inner == AC_INNER_EXACT) return 0;
    if (o->inner == AC_INNER_SP) return static_cast<long long>(pm[0]) * (2LL * (p->ell - p->nsr) + p->nsr);
    long long s = 0;
    for (int v : pm) s += v;
    return s;
}
// The paper's outer solver (Section 5): Chebyshev semi-iteration on P^{-1} calA with
// the Corollary 1 interval [1, mu^l/(mu^l - alpha)] and a zero-residual-norm stop.
// Residual form: r = b - calA x, z = P^{-1} r, d_0 = z/theta, x_{k+1} = x_k + d_k,
// rho_0 = delta/theta, rho_{k+1} = 1/(2 theta/delta - rho_k),
// d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) z_{k+1}.
int outer_cheb_impl(ac_problem* p, const ac_solve_opts* o, const std::vector<int>& pm, const double* b, double* x,
                    void* ws, ac_solve_info* info, std::chrono::steady_clock::time_point t0) {
    if (o->inner != AC_INNER_CHEB && o->inner != AC_INNER_EXACT && o->inner != AC_INNER_SP)
        return fail(AC_ERR_UNSUPPORTED, "the outer Chebyshev iteration takes the Chebyshev, exact or saddle-point "
                                        "inner solves");
    if (p->kblocks)
        return fail(AC_ERR_UNSUPPORTED, "no eigenvalue interval is known for varying diagonal blocks (use FGMRES)");
    // bf16 rounding of kappa (relative 2^-9) moves the eigenvalues of P^{-1} calA by more
    // than the width of the Corollary 1 interval at small alpha, and the iteration diverges
    if (o->precision == AC_PREC_MIXED_BF16K)
        return fail(AC_ERR_UNSUPPORTED, "the outer Chebyshev iteration needs float32 or float64 kappa in the inner solve");
    ac_ctx* c = p->ctx;
    hipStream_t st = c->stream;
    const long long len = static_cast<long long>(p->ell) * p->g.n;
    SolveWs w = carve_solve(p, o, ws);
    double* r = w.V[0];
    double* d = w.V[1];
    double* z = w.Z[0];
    const int kb = ac::krylov_blocks();
    const int ptiles = static_cast<int>(calA_partials(p));
    const long long psum = prec_products(p, o, pm);
    const double mul = std::pow(p->bounds[AC_PREC_FP64][0], p->ell);
    const double lo = 1.0, hi = mul / (mul - p->alpha);
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    auto fetch1 = [&](double& v) -> int {
        AC_HIP(hipMemcpyAsync(c->pinned, w.red, sizeof(double), hipMemcpyDeviceToHost, st));
        AC_HIP(hipStreamSynchronize(st));
        v = c->pinned[0];
        return AC_OK;
    };
    double bb = 0.0;
    {
        ProfScope ps(c, AC_K_KRYLOV, 8.0 * len);
        AC_HIP(ac::launch_norm2(b, len, w.partial, st));
        AC_HIP(ac::launch_reduce(w.partial, kb, 1, 1, w.red, st));
    }
    AC_TRY(fetch1(bb));
    const double bnorm = std::sqrt(bb);
    if (!std::isfinite(bnorm)) return fail(AC_ERR_NONFINITE, "b is not finite");
    if (bnorm == 0.0) {  // the solution is x = 0, whatever the initial guess
        AC_HIP(launch_zero(x, len, st));
        AC_HIP(hipStreamSynchronize(st));
        if (info) *info = ac_solve_info{};
        return AC_OK;
    }
    long long matvecs = 0;
    int it = 0, status = AC_OK;
    double beta = 0.0, rho = delta / theta;
    while (true) {
        AC_TRY(calA_impl(p, x, r, b, w.partial2));
        AC_HIP(ac::launch_reduce(w.partial2, ptiles, 1, 1, w.red, st));
        double rr = 0.0;
        AC_TRY(fetch1(rr));
        matvecs += p->ell;
        beta = std::sqrt(rr);
        if (!std::isfinite(beta)) return fail(AC_ERR_NONFINITE, "residual is not finite");
        if (beta / bnorm <= o->tol) break;
        if (it >= o->max_outer) {
            status = AC_NOT_CONVERGED;
            break;
        }
        AC_TRY(apply_prec_impl(p, o, pm, r, z, w.prec, 1.0));
        matvecs += psum;
        double a_k = 0.0, c_k = 1.0 / theta;
        if (it > 0 && delta > 0.0) {
            const double rn = 1.0 / (2.0 * theta / delta - rho);
            a_k = rn * rho;
            c_k = 2.0 * rn / delta;
            rho = rn;
        }
        ProfScope ps(c, AC_K_KRYLOV, 40.0 * len);
        AC_HIP(ac::launch_cheb_update(x, d, z, a_k, c_k, len, st));
        ++it;
    }
    // the residual evaluations count l products each; the paper counts l per
    // iteration, so drop the final check's product from the total
    if (it > 0) matvecs -= p->ell;
    if (info) {
        *info = ac_solve_info{};
        info->outer_iters = it;
        info->matvecs_A = matvecs;
        info->rel_residual_true = bnorm > 0 ? beta / bnorm : 0.0;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int solve_impl(ac_problem* p, const ac_solve_opts* o, const double* b, double* x, void* ws, size_t ws_bytes,
               ac_solve_info* info, double* rec, int rec_count, int* rec_done) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!p || !b || !x) return fail(AC_ERR_ARG, "NULL argument");
    if (ranges_overlap(b, x, block_bytes(p))) return fail(AC_ERR_ARG, "b and x overlap");
    std::vector<int> pm;
    AC_TRY(validate_opts(p, o, pm));
    if (o->restart_m < 1 || o->restart_m > 32) return fail(AC_ERR_UNSUPPORTED, "restart_m must be in [1, 32]");
    if (!(o->tol > 0.0)) return fail(AC_ERR_ARG, "tol must be positive");
    if (o->max_outer < 1) return fail(AC_ERR_ARG, "max_outer must be >= 1");
    if (o->outer != AC_OUTER_FGMRES && o->outer != AC_OUTER_CHEBYSHEV) return fail(AC_ERR_ARG, "unknown outer solver");
    if (!ws || ws_bytes < solve_ws_bytes(p, o)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(p->ctx->device));
    if (o->outer == AC_OUTER_CHEBYSHEV) {
        if (rec) return fail(AC_ERR_UNSUPPORTED, "recording needs the FGMRES outer solver");
        return outer_cheb_impl(p, o, pm, b, x, ws, info, t0);
    }
    ac_ctx* c = p->ctx;
    hipStream_t st = c->stream;
    const int m = o->restart_m;
    const long long len = static_cast<long long>(p->ell) * p->g.n;
    SolveWs w = carve_solve(p, o, ws);
    const int kb = ac::krylov_blocks();
    const int ptiles = static_cast<int>(calA_partials(p));
    const long long psum = prec_products(p, o, pm);
    long long matvecs = 0;

    auto fetch = [&](int nq) -> int {
        AC_HIP(hipMemcpyAsync(c->pinned, w.red, nq * sizeof(double), hipMemcpyDeviceToHost, st));
        AC_HIP(hipStreamSynchronize(st));
        return AC_OK;
    };
    // ||b||
    {
        ProfScope ps(c, AC_K_KRYLOV, 8.0 * len);
        AC_HIP(ac::launch_norm2(b, len, w.partial, st));
        AC_HIP(ac::launch_reduce(w.partial, kb, 1, 1, w.red, st));
    }
    AC_TRY(fetch(1));
    const double bnorm = std::sqrt(c->pinned[0]);
    if (!std::isfinite(bnorm)) return fail(AC_ERR_NONFINITE, "b is not finite");
    auto residual = [&](double& beta) -> int {
        AC_TRY(calA_impl(p, x, w.V[0], b, w.partial2));
        AC_HIP(ac::launch_reduce(w.partial2, ptiles, 1, 1, w.red, st));
        AC_TRY(fetch(1));
        beta = std::sqrt(c->pinned[0]);
        matvecs += p->ell;
        return AC_OK;
    };
    if (bnorm == 0.0) {
        AC_HIP(launch_zero(x, len, st));
        AC_HIP(hipStreamSynchronize(st));
        if (info) {
            *info = ac_solve_info{};
        }
        return AC_OK;
    }
    double beta = 0;
    AC_TRY(residual(beta));
    int total = 0, restarts = 0, fallbacks = 0;
    double orth_loss = 0.0;
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), scale(m + 1), y(m), Lg(m * m), hcol(m + 1);
    int status = AC_OK;
    while (true) {
        if (!std::isfinite(beta)) return fail(AC_ERR_NONFINITE, "residual is not finite");
        if (beta / bnorm <= o->tol) break;
        if (total >= o->max_outer) {
            status = AC_NOT_CONVERGED;
            break;
        }
        if (o->inner == AC_INNER_CHEB_CNN_MR) {
            // warm-started correction before the cycle: zw = P_warm(r) (the network's guesses
            // corrected by the Chebyshev steps), then the one-dimensional minimal-residual
            // step x += gamma zw, r -= gamma calA zw, gamma = <calA zw, r> / |calA zw|^2:
            // the residual never grows, and the cycle that follows is the plain method's
            ac_solve_opts ow = *o;
            ow.inner = AC_INNER_CHEB_CNN;
            AC_TRY(apply_prec_impl(p, &ow, pm, w.V[0], w.Z[0], w.prec, 1.0 / beta, &fallbacks));
            AC_TRY(calA_impl(p, w.Z[0], w.V[1], nullptr, nullptr));
            matvecs += p->ell + psum;
            {
                ProfScope ps(c, AC_K_KRYLOV, 8.0 * len * 2);
                AC_HIP(ac::launch_mdot_strided(w.V[0], static_cast<long long>(vec_bytes(p) / sizeof(double)), 1,
                                               false, w.V[1], len, w.partial, 72, st));
                AC_HIP(ac::launch_reduce(w.partial, kb, 2, 72, w.red, st));
            }
            AC_TRY(fetch(2));
            const double wr = c->pinned[0], ww = c->pinned[1];
            if (ww > 0.0 && std::isfinite(wr) && std::isfinite(ww)) {
                const double gam = wr / ww;
                ac::VecSet zs{}, ws1{};
                zs.v[0] = w.Z[0];
                zs.s2[0] = gam;
                ws1.v[0] = w.V[1];
                ws1.s2[0] = gam;
                {
                    ProfScope ps(c, AC_K_KRYLOV, 8.0 * len * 3);
                    AC_HIP(ac::launch_maxpy(zs, 1, nullptr, x, len, st));
                }
                {
                    ProfScope ps(c, AC_K_KRYLOV, 8.0 * len * 3);
                    AC_HIP(ac::launch_axpy_norm(ws1, 1, nullptr, w.V[0], len, w.partial, 72, st));
                    AC_HIP(ac::launch_reduce(w.partial, kb, 1, 72, w.red, st));
                }
                AC_TRY(fetch(1));
                beta = std::sqrt(c->pinned[0]);
                if (!std::isfinite(beta)) return fail(AC_ERR_NONFINITE, "residual is not finite");
                if (beta / bnorm <= o->tol) break;
            }
        }
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        scale[0] = 1.0 / beta;
        int kdone = 0;
        // the transform of V_j is already in the preconditioner workspace (made by the
        // previous step's fused Gram-Schmidt update, unscaled)
        bool rhat_ready = false;
        for (int j = 0; j < m; ++j) {
            if (rec && *rec_done < rec_count) {
                AC_HIP(hipMemcpyAsync(rec + static_cast<size_t>(*rec_done) * len, w.V[j], len * sizeof(double),
                                      hipMemcpyDeviceToDevice, st));
                ++*rec_done;
            }
            // z_j = P^{-1} v_j with v_j = scale_j * V_j (scale folded into the transform);
            // AC_INNER_CHEB_CNN_CYCLE warm-starts only the cycle's first vector
            ac_solve_opts oj = *o;
            if ((o->inner == AC_INNER_CHEB_CNN_CYCLE && j > 0) || o->inner == AC_INNER_CHEB_CNN_MR)
                oj.inner = AC_INNER_CHEB;
            if (rhat_ready) AC_TRY(apply_prec_rhat(p, &oj, pm, w.Z[j], w.prec, scale[j]));
            else AC_TRY(apply_prec_impl(p, &oj, pm, w.V[j], w.Z[j], w.prec, scale[j], &fallbacks));
            rhat_ready = false;
            AC_TRY(calA_impl(p, w.Z[j], w.V[j + 1], nullptr, nullptr));
            matvecs += p->ell + psum;
            ac::VecSet vs{};
            for (int i = 0; i <= j; ++i) vs.v[i] = w.V[i];
            const int nv = j + 1;
            // Modified Gram-Schmidt in inverse compact WY form (one reduction per step):
            // the projector (I - q_j q_j^T)...(I - q_0 q_0^T) equals I - Q (I + L)^{-1} Q^T with
            // L the strictly lower part of Q^T Q.  One sweep gives r = Q^T w and the new row
            // of L (dots of the newest basis vector with the older ones); the host solves
            // (I + L) h = r; a second sweep forms w - Q h and its norm.
            {
                ProfScope ps(c, AC_K_KRYLOV, 8.0 * len * (nv + 1));
                AC_HIP(ac::launch_mdot_strided(w.V[0], static_cast<long long>(vec_bytes(p) / sizeof(double)), nv,
                                               j >= 1, w.V[j + 1], len, w.partial, 72, st));
                AC_HIP(ac::launch_reduce(w.partial, kb, j >= 1 ? 2 * nv : nv + 1, 72, w.red, st));
            }
            AC_TRY(fetch(2 * nv + 1));
            {
                const double* hd = c->pinned;
                for (int i = 0; i < j; ++i) {
                    Lg[j * m + i] = scale[i] * scale[j] * hd[nv + 1 + i];
                    orth_loss = std::max(orth_loss, std::abs(Lg[j * m + i]));
                }
                for (int i = 0; i <= j; ++i) {
                    double hi = scale[i] * hd[i];
                    for (int k = 0; k < i; ++k) hi -= Lg[i * m + k] * hcol[k];
                    hcol[i] = hi;
                    H[i * m + j] = hi;
                    vs.s2[i] = scale[i] * hi;  // coefficient of the raw basis vector
                }
            }
            // the next step's preconditioner input V_{j+1} is formed here; when that step
            // applies the plain nested Chebyshev, its forward transform is computed in the
            // same pass (the norm, known only afterwards, scales the result instead)
            const bool fuse_fwd = j + 1 < m && prec_from_rhat_ok(p, o);
            if (fuse_fwd) {
                int nblk = 0;
                AC_TRY(axpy_fwd_impl(p, o, vs, nv, w.V[j + 1], w.prec, w.partial, 72, &nblk));
                AC_HIP(ac::launch_reduce(w.partial, nblk, 1, 72, w.red, st));
            } else {
                ProfScope ps(c, AC_K_KRYLOV, 8.0 * len * (nv + 2));
                AC_HIP(ac::launch_axpy_norm(vs, nv, nullptr, w.V[j + 1], len, w.partial, 72, st));
                AC_HIP(ac::launch_reduce(w.partial, kb, 1, 72, w.red, st));
            }
            AC_TRY(fetch(1));
            const double hn = std::sqrt(c->pinned[0]);
            if (!std::isfinite(hn)) return fail(AC_ERR_NONFINITE, "Arnoldi produced a non-finite value");
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t;
            }
            const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
            cs[j] = den > 0 ? H[j * m + j] / den : 1.0;
            sn[j] = den > 0 ? H[(j + 1) * m + j] / den : 0.0;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            kdone = j + 1;
            if (std::abs(g[j + 1]) / bnorm <= o->tol || total >= o->max_outer || hn == 0.0) break;
            scale[j + 1] = 1.0 / hn;
            rhat_ready = fuse_fwd;
        }
        // back substitution and x += Z y
        for (int i = kdone - 1; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k < kdone; ++k) t -= H[i * m + k] * y[k];
            y[i] = H[i * m + i] != 0.0 ? t / H[i * m + i] : 0.0;
        }
        {
            ac::VecSet zs{};
            for (int i = 0; i < kdone; ++i) {
                zs.v[i] = w.Z[i];
                zs.s2[i] = y[i];
            }
            ProfScope ps(c, AC_K_KRYLOV, 8.0 * len * (kdone + 2));
            AC_HIP(ac::launch_maxpy(zs, kdone, nullptr, x, len, st));
        }
        ++restarts;
        AC_TRY(residual(beta));
    }
    if (info) {
        info->outer_iters = total;
        info->restarts = restarts;
        info->matvecs_A = matvecs;
        info->rel_residual_true = beta / bnorm;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->cnn_fallbacks = fallbacks;
        info->reserved = 0;
        info->orth_loss = orth_loss;
    }
    if (rec) AC_HIP(hipStreamSynchronize(st));
    return status;
}
}  // namespace

int ac_solve(ac_problem* p, const ac_solve_opts* o, const double* b, double* x, void* ws, size_t ws_bytes,
             ac_solve_info* info) {
    return solve_impl(p, o, b, x, ws, ws_bytes, info, nullptr, 0, nullptr);
}

int ac_solve_record(ac_problem* p, const ac_solve_opts* o, const double* b, double* x, void* ws, size_t ws_bytes,
                    ac_solve_info* info, double* rec, int rec_count, int* recorded) {
    if (!rec || rec_count < 1 || !recorded) return fail(AC_ERR_ARG, "record buffer, count and counter are required");
    *recorded = 0;
    return solve_impl(p, o, b, x, ws, ws_bytes, info, rec, rec_count, recorded);
}
