// C ABI of alphacirc: batched solves of many independent problems, one captured
// FGMRES cycle of all problems at a time.
#include "host.h"

using namespace ach;

// ---------------------------------------------------------------------------
// Batched solves: many independent problems (uneven grids and l) advance their
// FGMRES iterations in lockstep.  Per Arnoldi index j the preconditioner and the
// calA product of every problem are recorded once as launch records, and aligned
// records are grouped by kernel variant into work lists; so is the residual
// b - calA x.  The Arnoldi scalars of every problem (Gram-Schmidt coefficients,
// Givens rotations, convergence and restart tests) live in device memory and are
// updated by small kernels, so one whole FGMRES cycle of all problems is captured
// once as a hipGraph and replayed; the host reads one counter per cycle.

namespace {

constexpr int kMaxBatch = 256;
constexpr int kFetchStride = 2 * ac::kMaxBasis + 2;  // pinned doubles per problem per fetch

struct BatchLaunch {
    int op, ell, prec, curk, vx;
    ac::BatchList list;
};

size_t max_args_bytes() {
    return std::max({sizeof(ac::SweepArgs<double>), sizeof(ac::SweepArgs<float>), sizeof(ac::FwdArgs),
                     sizeof(ac::CalAArgs), sizeof(ac::TripleArgs<double>), sizeof(ac::TripleArgs<float>),
                     sizeof(ac::PairArgs<double>), sizeof(ac::PairArgs<float>)});
}

// Device bytes for the work lists: per j (and once more for the residual form) at most
// kMaxGroups p + 3 launch positions (a sweep step records kMaxGroups shift groups),
// each with at most `count` groups.
size_t batch_list_bytes(int count, const ac_solve_opts* o) {
    const size_t per_pos = static_cast<size_t>(count) * (align_up(max_args_bytes(), 16) + 8) +
                           static_cast<size_t>(count) * (3 * 256 + 8);
    return static_cast<size_t>(o->restart_m + 1) * static_cast<size_t>(kMaxGroups * o->p_uniform + 3) * per_pos + 256;
}

size_t batch_kry_bytes(int count) {
    return align_up(static_cast<size_t>(count + 1) * sizeof(int), 256) +
           align_up(static_cast<size_t>(count) * sizeof(ac::BKProb), 256) +
           align_up(static_cast<size_t>(count) * sizeof(ac::BKState), 256);
}

size_t batch_ws_bytes(int count, ac_problem* const* probs, const ac_solve_opts* o) {
    size_t b = batch_list_bytes(count, o) + align_up(static_cast<size_t>(count) * 12, 256) + 256 +
               batch_kry_bytes(count);
    for (int q = 0; q < count; ++q) b += align_up(solve_ws_bytes(probs[q], o), 256);
    return b;
}

int validate_batch(ac_ctx* c, int count, ac_problem* const* probs, const ac_solve_opts* o) {
    if (!c || !probs || !o) return fail(AC_ERR_ARG, "NULL argument");
    if (count < 1 || count > kMaxBatch) return fail(AC_ERR_UNSUPPORTED, "batch size must be in [1, 256]");
    if (o->inner != AC_INNER_CHEB) return fail(AC_ERR_UNSUPPORTED, "batched solves use the plain inner solver");
    if (o->outer != AC_OUTER_FGMRES) return fail(AC_ERR_UNSUPPORTED, "batched solves use the FGMRES outer solver");
    if (o->p_per_shift) return fail(AC_ERR_UNSUPPORTED, "batched solves take a uniform inner count (p_uniform)");
    if (o->restart_m < 1 || o->restart_m > 32) return fail(AC_ERR_UNSUPPORTED, "restart_m must be in [1, 32]");
    if (!(o->tol > 0.0)) return fail(AC_ERR_ARG, "tol must be positive");
    if (o->max_outer < 1) return fail(AC_ERR_ARG, "max_outer must be >= 1");
    for (int q = 0; q < count; ++q) {
        if (!probs[q]) return fail(AC_ERR_ARG, "NULL problem");
        if (probs[q]->ctx != c) return fail(AC_ERR_ARG, "every problem must belong to the context");
        if (probs[q]->g.periodic) return fail(AC_ERR_UNSUPPORTED, "batched solves take Dirichlet grids");
        if (probs[q]->kblocks) return fail(AC_ERR_UNSUPPORTED, "batched solves take one block operator per problem");
        std::vector<int> pm;
        AC_TRY(validate_opts(probs[q], o, pm));
    }
    return AC_OK;
}

struct BatchState {
    ac_problem* p;
    SolveWs w;
    std::vector<int> pm;
    long long len = 0, psum = 0;
};

// Restores the context and frees the graphs and the capture stream on every exit path.
struct BatchGuard {
    ac_ctx* c;
    hipStream_t user, own = nullptr;
    bool prof;
    std::vector<hipGraphExec_t> execs;
    ~BatchGuard() {
        c->rec = nullptr;
        if (own) (void)hipStreamSynchronize(own);
        for (auto e : execs)
            if (e) (void)hipGraphExecDestroy(e);
        if (own) (void)hipStreamDestroy(own);
        c->stream = user;
        c->profiling = prof;
    }
};

}  // namespace

int ac_batch_workspace_size(ac_ctx* c, int count, ac_problem* const* probs, const ac_solve_opts* o,
                            size_t* bytes) {
    if (!bytes) return fail(AC_ERR_ARG, "NULL argument");
    AC_TRY(validate_batch(c, count, probs, o));
    *bytes = batch_ws_bytes(count, probs, o);
    return AC_OK;
}

int ac_batch_solve(ac_ctx* c, int count, ac_problem* const* probs, const ac_solve_opts* o, const double* const* b,
                   double* const* x, void* ws, size_t ws_bytes, ac_solve_info* infos) {
    const auto t0 = std::chrono::steady_clock::now();
    AC_TRY(validate_batch(c, count, probs, o));
    if (!b || !x) return fail(AC_ERR_ARG, "NULL argument");
    for (int q = 0; q < count; ++q) {
        if (!b[q] || !x[q]) return fail(AC_ERR_ARG, "NULL right-hand side or solution");
        if (ranges_overlap(b[q], x[q], block_bytes(probs[q]))) return fail(AC_ERR_ARG, "b and x overlap");
    }
    if (!ws || ws_bytes < batch_ws_bytes(count, probs, o)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(c->device));
    const int m = o->restart_m;
    // The legacy default stream cannot be captured: work on a stream of our own.
    AC_HIP(hipStreamSynchronize(c->stream));
    BatchGuard guard{c, c->stream, nullptr, c->profiling, std::vector<hipGraphExec_t>(1, nullptr)};
    AC_HIP(hipStreamCreateWithFlags(&guard.own, hipStreamNonBlocking));
    hipStream_t st = guard.own;
    c->stream = st;
    c->profiling = false;

    // workspace: [lists][scale doubles | live ints][cycle mask, active count | problem
    // list | scalar states][per-problem solve workspaces]
    char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(ws), 256));
    char* lists = base;
    const size_t list_cap = batch_list_bytes(count, o);
    double* dscale = reinterpret_cast<double*>(base + align_up(list_cap, 256));
    int* dlive = reinterpret_cast<int*>(dscale + count);
    char* pw = base + align_up(list_cap, 256) + align_up(static_cast<size_t>(count) * 12, 256) +
               batch_kry_bytes(count);
    std::vector<BatchState> S(count);
    for (int q = 0; q < count; ++q) {
        BatchState& s = S[q];
        s.p = probs[q];
        AC_TRY(validate_opts(s.p, o, s.pm));
        s.w = carve_solve(s.p, o, pw);
        pw += align_up(solve_ws_bytes(s.p, o), 256);
        s.len = static_cast<long long>(s.p->ell) * s.p->g.n;
        for (int v : s.pm) s.psum += v;
    }

    // record every problem's launches for each j (and the residual form) and group
    // aligned records into work lists
    std::vector<std::vector<BatchLaunch>> plan(m + 1);  // plan[m]: the residual b - calA x
    std::vector<char> host(list_cap, 0);
    size_t used = 0;
    auto take = [&](size_t bytes, size_t align) -> size_t {
        used = align_up(used, align);
        const size_t off = used;
        used += bytes;
        return off;
    };
    struct Pending {
        BatchLaunch l;
        size_t args_off, first_off, pid_off;
    };
    std::vector<std::vector<Pending>> pend(m + 1);
    auto group = [&](std::vector<std::vector<ac_launch_rec>>& recs, std::vector<Pending>& out) -> int {
        for (int q = 0; q < count; ++q)
            if (recs[q].size() != recs[0].size()) return fail(AC_ERR_UNSUPPORTED, "batch launch sequences differ");
        const size_t npos = recs[0].size();
        for (size_t i = 0; i < npos; ++i) {
            std::vector<int> done(count, 0);
            for (int q = 0; q < count; ++q) {
                if (recs[q][i].op != recs[0][i].op) return fail(AC_ERR_UNSUPPORTED, "batch launch sequences differ");
                if (recs[q][i].blocks == 0) done[q] = 1;  // an empty shift group
            }
            for (int q0 = 0; q0 < count; ++q0) {
                if (done[q0]) continue;
                const ac_launch_rec& r0 = recs[q0][i];
                std::vector<int> members;
                for (int q = q0; q < count; ++q) {
                    const ac_launch_rec& r = recs[q][i];
                    if (!done[q] && r.ell == r0.ell && r.prec == r0.prec && r.curk == r0.curk && r.vx == r0.vx &&
                        r.wpb == r0.wpb) {
                        members.push_back(q);
                        done[q] = 1;
                    }
                }
                const size_t asz = r0.args.size();
                Pending pg{};
                pg.l = BatchLaunch{r0.op, r0.ell, r0.prec, r0.curk, r0.vx, ac::BatchList{}};
                const int n = static_cast<int>(members.size());
                pg.args_off = take(asz * n, 256);
                pg.first_off = take(sizeof(int) * (n + 1), 16);
                pg.pid_off = take(sizeof(int) * n, 16);
                if (used > list_cap) return fail(AC_ERR_WORKSPACE, "batch work lists exceed their bound");
                int* first = reinterpret_cast<int*>(host.data() + pg.first_off);
                int* pid = reinterpret_cast<int*>(host.data() + pg.pid_off);
                int blocks = 0;
                for (int k = 0; k < n; ++k) {
                    const ac_launch_rec& r = recs[members[k]][i];
                    std::memcpy(host.data() + pg.args_off + asz * k, r.args.data(), asz);
                    first[k] = blocks;
                    pid[k] = members[k];
                    blocks += r.blocks;
                }
                first[n] = blocks;
                pg.l.list.nprob = n;
                pg.l.list.blocks = blocks;
                pg.l.list.wpb = r0.wpb;
                out.push_back(pg);
            }
        }
        return AC_OK;
    };
    for (int j = 0; j <= m; ++j) {
        std::vector<std::vector<ac_launch_rec>> recs(count);
        for (int q = 0; q < count; ++q) {
            BatchState& s = S[q];
            c->rec = &recs[q];
            int e = AC_OK;
            if (j < m) {
                e = apply_prec_impl(s.p, o, s.pm, s.w.V[j], s.w.Z[j], s.w.prec, 1.0);
                if (e >= 0) e = calA_impl(s.p, s.w.Z[j], s.w.V[j + 1], nullptr, nullptr);
            } else {
                e = calA_impl(s.p, x[q], s.w.V[0], b[q], s.w.partial2);
            }
            c->rec = nullptr;
            if (e < 0) return e;
        }
        AC_TRY(group(recs, pend[j]));
    }

    // device state of the batched FGMRES: problem list, scalar states, masks
    char* kry = base + align_up(list_cap, 256) + align_up(static_cast<size_t>(count) * 12, 256);
    int* dcyc = reinterpret_cast<int*>(kry);
    ac::BKProb* dP = reinterpret_cast<ac::BKProb*>(kry + align_up(static_cast<size_t>(count + 1) * sizeof(int), 256));
    ac::BKState* dS = reinterpret_cast<ac::BKState*>(reinterpret_cast<char*>(dP) +
                                                     align_up(static_cast<size_t>(count) * sizeof(ac::BKProb), 256));
    std::vector<ac::BKProb> hP(count);
    int kblocks = 0;
    for (int q = 0; q < count; ++q) {
        BatchState& s = S[q];
        ac::BKProb& bp = hP[q];
        bp.v0 = s.w.V[0];
        bp.z0 = s.w.Z[0];
        bp.x = x[q];
        bp.vstride = static_cast<long long>(vec_bytes(s.p) / sizeof(double));
        bp.len = s.len;
        bp.partial = s.w.partial;
        bp.partial2 = s.w.partial2;
        bp.ntiles = static_cast<int>(calA_partials(s.p));
        // one block per 512 elements, at most the single solve's block count
        const long long want = (s.len + 511) / 512;
        bp.nblk = static_cast<int>(std::min<long long>(std::max<long long>(want, 1), ac::krylov_blocks()));
        kblocks += bp.nblk;
    }
    AC_HIP(hipMemcpyAsync(dP, hP.data(), static_cast<size_t>(count) * sizeof(ac::BKProb), hipMemcpyHostToDevice, st));
    AC_HIP(hipMemcpyAsync(lists, host.data(), used, hipMemcpyHostToDevice, st));
    for (int j = 0; j <= m; ++j)
        for (auto& pg : pend[j]) {
            BatchLaunch l = pg.l;
            l.list.args = lists + pg.args_off;
            l.list.first = reinterpret_cast<const int*>(lists + pg.first_off);
            l.list.pid = reinterpret_cast<const int*>(lists + pg.pid_off);
            l.list.live = j < m ? dlive : dcyc;
            l.list.scale = l.op == ac::BOP_FWD ? dscale : nullptr;
            plan[j].push_back(l);
        }

    auto fetch = [&](const std::vector<int>& qs, int nq) -> int {
        for (int q : qs)
            AC_HIP(hipMemcpyAsync(c->pinned + static_cast<size_t>(q) * kFetchStride, S[q].w.red,
                                  nq * sizeof(double), hipMemcpyDeviceToHost, st));
        AC_HIP(hipStreamSynchronize(st));
        return AC_OK;
    };
    auto fetched = [&](int q) { return c->pinned + static_cast<size_t>(q) * kFetchStride; };
    const int kb = ac::krylov_blocks();

    // ||b|| and the first residuals (once, on the host)
    std::vector<int> all(count);
    for (int q = 0; q < count; ++q) {
        all[q] = q;
        AC_HIP(ac::launch_norm2(b[q], S[q].len, S[q].w.partial, st));
        AC_HIP(ac::launch_reduce(S[q].w.partial, kb, 1, 1, S[q].w.red, st));
    }
    AC_TRY(fetch(all, 1));
    std::vector<int> live_q;
    std::vector<ac::BKState> hS(count);
    for (int q = 0; q < count; ++q) {
        ac::BKState& ks = hS[q];
        std::memset(&ks, 0, sizeof(ks));
        ks.ell = S[q].p->ell;
        ks.psum = S[q].psum;
        ks.bnorm = std::sqrt(fetched(q)[0]);
        if (!std::isfinite(ks.bnorm)) return fail(AC_ERR_NONFINITE, "b is not finite");
        if (ks.bnorm == 0.0) {
            AC_HIP(launch_zero(x[q], S[q].len, st));
            ks.finished = 1;
        } else {
            live_q.push_back(q);
        }
    }
    for (int q : live_q) {
        BatchState& s = S[q];
        AC_TRY(calA_impl(s.p, x[q], s.w.V[0], b[q], s.w.partial2));
        AC_HIP(ac::launch_reduce(s.w.partial2, static_cast<int>(calA_partials(s.p)), 1, 1, s.w.red, st));
    }
    AC_TRY(fetch(live_q, 1));
    for (int q : live_q) {
        hS[q].beta = std::sqrt(fetched(q)[0]);
        hS[q].matvecs = S[q].p->ell;
    }
    AC_HIP(hipMemcpyAsync(dS, hS.data(), static_cast<size_t>(count) * sizeof(ac::BKState), hipMemcpyHostToDevice, st));
    AC_HIP(launch_zero_int(dcyc, count, st));
    AC_HIP(ac::launch_bk_cycle(dP, dS, count, dlive, dcyc, dscale, m, o->tol, o->max_outer, st));
    // problems in the next cycle, read from the cycle mask
    int* hcyc = reinterpret_cast<int*>(c->pinned);
    auto active = [&]() -> int {
        AC_HIP(hipMemcpyAsync(hcyc, dcyc, static_cast<size_t>(count) * sizeof(int), hipMemcpyDeviceToHost, st));
        AC_HIP(hipStreamSynchronize(st));
        int n = 0;
        for (int q = 0; q < count; ++q) n += hcyc[q] != 0;
        return n;
    };
    int nact = active();
    if (nact < 0) return nact;

    // One FGMRES cycle of every problem in it, captured once as a graph: per Arnoldi
    // index the preconditioner and calA work lists, the batched multi-dot, the
    // Gram-Schmidt coefficients, the multi-axpy with the new norm and the Givens update;
    // then x += Z y, the residuals, and the restart test that sets the next cycle's
    // masks.  The host reads one counter per cycle.
    auto record_cycle = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int j = 0; j < m && e == hipSuccess; ++j) {
            for (const BatchLaunch& l : plan[j]) {
                e = ac::launch_batch(l.op, l.ell, l.prec, l.curk, l.vx, l.list, st);
                if (e != hipSuccess) return e;
            }
            const int nv = j + 1;
            e = ac::launch_bk_mdot(dP, count, kblocks, dlive, nv, st);
            if (e == hipSuccess) e = ac::launch_bk_arnoldi(dP, dS, count, dlive, j, m, st);
            if (e == hipSuccess) e = ac::launch_bk_axpy_norm(dP, dS, count, kblocks, dlive, nv, st);
            if (e == hipSuccess) e = ac::launch_bk_givens(dP, dS, count, dlive, dscale, j, m, o->tol, o->max_outer, st);
        }
        if (e == hipSuccess) e = ac::launch_bk_update(dP, dS, count, kblocks, dcyc, m, st);
        for (const BatchLaunch& l : plan[m]) {
            if (e != hipSuccess) break;
            e = ac::launch_batch(l.op, l.ell, l.prec, l.curk, l.vx, l.list, st);
        }
        if (e == hipSuccess) e = ac::launch_bk_cycle(dP, dS, count, dlive, dcyc, dscale, m, o->tol, o->max_outer, st);
        return e;
    };
    while (nact > 0) {
        if (!guard.execs[0]) {
            AC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const hipError_t le = record_cycle();
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(st, &graph);
            if (le != hipSuccess || ee != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(AC_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ee));
            }
            const hipError_t ie = hipGraphInstantiate(&guard.execs[0], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(AC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        }
        AC_HIP(hipGraphLaunch(guard.execs[0], st));
        nact = active();
        if (nact < 0) return nact;
    }
    AC_HIP(hipMemcpyAsync(hS.data(), dS, static_cast<size_t>(count) * sizeof(ac::BKState), hipMemcpyDeviceToHost, st));
    AC_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = AC_OK;
    for (int q = 0; q < count; ++q) {
        const ac::BKState& ks = hS[q];
        if (ks.status == AC_ERR_NONFINITE) return fail(AC_ERR_NONFINITE, "a batched solve produced a non-finite value");
        if (ks.status == AC_NOT_CONVERGED) worst = AC_NOT_CONVERGED;
        if (!infos) continue;
        ac_solve_info& in = infos[q];
        in = ac_solve_info{};
        in.outer_iters = ks.total;
        in.restarts = ks.restarts;
        in.matvecs_A = ks.matvecs;
        in.rel_residual_true = ks.bnorm > 0 ? ks.beta / ks.bnorm : 0.0;
        in.seconds = secs;
        in.orth_loss = ks.orth;
    }
    return worst;
}
