// C ABI of alphacirc, first part: contexts, problems and the preconditioner stages
// (the outer solves, batches, tuner and network are in solve.hip, batch.hip,
// tuner.hip and cnn_api.hip).  Host orchestration only; every vector operation runs
// in the kernels behind ac_internal.h.
#include "host.h"

using namespace ach;

// ---------------------------------------------------------------------------
// error plumbing

namespace ach {
thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

}  // namespace ach

int ac::set_error(int status, const std::string& msg) { return ach::fail(status, msg); }

namespace ach {

constexpr double kPi = 3.14159265358979323846;

}  // namespace ach

// ---------------------------------------------------------------------------
// opaque-type accessors for the kernel units

int ac::problem_device(const ac_problem* p) { return p->ctx->device; }
int ac::ctx_device(const ac_ctx* c) { return c->device; }
hipStream_t ac::ctx_stream(const ac_ctx* c) { return c->stream; }

// ---------------------------------------------------------------------------
// profiling helpers

namespace ach {


int harvest(ac_ctx* c) {
    AC_HIP(hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        float ms = 0.f;
        AC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        c->ms[p.cls] += ms;
        c->launches[p.cls] += p.launches;
        c->bytes[p.cls] += p.bytes;
        c->pool.emplace_back(p.a, p.b);
    }
    c->pending.clear();
    return AC_OK;
}

// ---------------------------------------------------------------------------
// geometry helpers

// Shift slot <-> frequency m.  Slot order: real shifts (m = 0, then m = l/2 for
// even l), then complex shifts m = 1..ceil(l/2)-1.
int slot_to_m(const ac_problem* p, int slot) {
    if (slot < p->nsr) return slot == 0 ? 0 : p->ell / 2;
    return slot - p->nsr + 1;
}
bool slot_is_real(const ac_problem* p, int slot) { return slot < p->nsr; }

size_t inner_elem(int prec) { return prec == AC_PREC_FP64 ? sizeof(double) : sizeof(float); }

// Elements (of the inner real type) of the slice for frequency m, padded.
long long slice_elems(const ac_problem* p, int m) {
    const bool real = (m == 0) || (p->ell % 2 == 0 && m == p->ell / 2);
    const long long e = real ? p->g.n : 2 * p->g.n;
    return (e + 63) / 64 * 64;
}

// True when the device ranges [a, a + bytes) and [b, b + bytes) intersect.
bool ranges_overlap(const void* a, const void* b, size_t bytes) {
    const auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

size_t block_bytes(const ac_problem* p) { return static_cast<size_t>(p->ell) * p->g.n * sizeof(double); }

// Kernels address block vectors and spectral buffers (l*N values, each slice padded to
// 64) with 32-bit element offsets: keep the padded total below 2^31.
bool block_elems_too_large(long long n, int ell) {
    return n * ell + 64LL * (ell / 2 + 1) > (1LL << 31) - 1;
}

// offsets by frequency m = 0..ns-1 (ABI order), last entry = total
void spectral_offsets(const ac_problem* p, long long* off) {
    long long o = 0;
    for (int m = 0; m < p->ns; ++m) {
        off[m] = o;
        o += slice_elems(p, m);
    }
    off[p->ns] = o;
}


bool use_shift_groups(const ac_problem* p) {
    const int mode = p->ctx->shift_groups;
    if (mode == 0) return false;
    return mode == 1 ? p->ns >= 2 : p->ns >= 5;
}

Tiling make_tiling(const ac_problem* p, int vx_pref, int h_pref, int wpb_pref) {
    Tiling t{};
    const Geom& g = p->g;
    int vx = vx_pref > 0 ? vx_pref : 2;
    if (g.nx % 2 != 0 || g.nx < 128 || g.periodic) vx = 1;  // periodic sweeps use one point per lane
    t.vx = vx;
    t.h = h_pref > 0 ? h_pref : (use_shift_groups(p) ? 8 : 16);
    if (t.h > g.ny) t.h = g.ny;
    t.wpb = wpb_pref > 0 ? wpb_pref : 4;
    t.nsx = (g.nx + ac::kWave * vx - 1) / (ac::kWave * vx);
    t.ncy = (g.ny + t.h - 1) / t.h;
    t.tiles = static_cast<long long>(t.nsx) * t.ncy;
    t.blocks = static_cast<int>((t.tiles + t.wpb - 1) / t.wpb);
    return t;
}

Tiling sweep_tiling(const ac_problem* p) {
    return make_tiling(p, p->tile_vx ? p->tile_vx : p->ctx->tile_vx, p->tile_h ? p->tile_h : p->ctx->tile_h,
                       p->tile_wpb ? p->tile_wpb : p->ctx->tile_wpb);
}

// Tiling of a fused block of `depth` steps (2 or 3): strips of 64*vx computed columns at
// a stride of 64*vx - 2*(depth-1); two points per lane on even grids at least 128 wide
// in float32, one in float64 (register budget); automatic height for about one round of
// waves at `occ` waves per SIMD.
Tiling block_tiling(const ac_problem* p, int prec, int depth, int h_pref, int wpb_pref, int vx_pref, int occ) {
    const Geom& g = p->g;
    Tiling t{};
    int vx = vx_pref > 0 ? vx_pref : (prec == AC_PREC_FP64 ? 1 : 2);
    if (g.nx % 2 != 0 || g.nx < 128) vx = 1;
    t.vx = vx;
    t.wpb = wpb_pref > 0 ? wpb_pref : 4;
    const int stride = ac::kWave * vx - 2 * (depth - 1);
    const int inner = g.nx - (depth - 1);  // columns past the first strip's low ghost edge
    t.nsx = (inner + stride - 1) / stride;
    const long long slots = static_cast<long long>(occ) * 1024;
    const int h = static_cast<int>((static_cast<long long>(t.nsx) * g.ny + slots - 1) / slots);
    t.h = h_pref > 0 ? h_pref : std::min(32, std::max(4, h));
    if (t.h > g.ny) t.h = g.ny;
    t.ncy = (g.ny + t.h - 1) / t.h;
    t.tiles = static_cast<long long>(t.nsx) * t.ncy;
    t.blocks = static_cast<int>((t.tiles + t.wpb - 1) / t.wpb);
    return t;
}

Tiling triple_tiling(const ac_problem* p, int prec, int groups) {
    const ac_ctx* c = p->ctx;
    return ac::triple_tiling(p->g, prec == AC_PREC_FP64, groups, c->triple_h, c->triple_vx, c->triple_occ);
}

// (the automatic height of the paired sweep, about one round of waves at three per
// SIMD, measured best at 2048^2: 12 rows, 96 us per launch against 100-103 us at 8 rows
// and 110 us at 16)
Tiling pair_tiling(const ac_problem* p, int prec) {
    const ac_ctx* c = p->ctx;
    return block_tiling(p, prec, 2, c->pair_h, c->pair_wpb, c->pair_vx, 3);
}

template <class A>
void record_launch(ac_ctx* c, int op, int ell, int prec, int curk, int vx, int wpb, int blocks, const A& a) {
    ac_launch_rec r{op, ell, prec, curk, vx, wpb, blocks, std::vector<char>(sizeof(A))};
    std::memcpy(r.args.data(), &a, sizeof(A));
    c->rec->push_back(std::move(r));
}

Tiling calA_tiling(const ac_problem* p) {
    if (p->kblocks || !ac::calA_strips(p->g)) {
        // halo-load form, float64 operand with l blocks per point: one point per lane
        // past l = 8
        return make_tiling(p, p->ell > 8 ? 1 : 2, 16, 4);
    }
    // overlapping strips: 64*vx - 2*vx owned columns per strip, 4-row chunks marching
    // down and up alternately (measured side by side at 2048^2, l = 10 over a whole
    // solve, two points per lane: 4 rows 0.5406 s, 8 rows 0.5416 s, 12 rows 0.5462 s,
    // 16 rows 0.5460 s; one point per lane and 8 rows 0.5469 s)
    Tiling t = make_tiling(p, p->ell > 12 ? 1 : 2, 4, 4);
    const int owned = ac::kWave * t.vx - 2 * t.vx;
    t.nsx = (p->g.nx + owned - 1) / owned;
    t.tiles = static_cast<long long>(t.nsx) * t.ncy;
    t.blocks = static_cast<int>((t.tiles + t.wpb - 1) / t.wpb);
    return t;
}

// ---------------------------------------------------------------------------
// Chebyshev tables (Section 3; textbook three-term recurrence in x form):
//   theta = (mu_hi + mu_lo)/2 - lambda, delta = (mu_hi - mu_lo)/2,
//   rho_0 = delta/theta, rho_k = 1/(2 theta/delta - rho_{k-1}),
//   x_{k+1} = x_k + rho_k rho_{k-1} (x_k - x_{k-1}) + (2 rho_k/delta)(rhat - B x_k),
//   x_1 = x_0 + (rhat - B x_0)/theta.
// lambda_m = alpha^{1/l} exp(-2 pi i m / l): the eigenvalue of C_alpha on the m-th
// column of the (negative-exponent) DFT that the forward transform applies.
cplx shift_of(const ac_problem* p, int m) { return std::polar(std::pow(p->alpha, 1.0 / p->ell), -2.0 * kPi * m / p->ell); }

struct ChebShift {
    cplx lam, theta;
    double delta;
    std::vector<cplx> a, c;  // index k = 0..p-1: coefficients producing x_{k+1}
};

ChebShift cheb_tables(const ac_problem* p, int prec, int m, int steps) {
    ChebShift s;
    const double lo = p->bounds[prec][0], hi = p->bounds[prec][1];
    s.lam = shift_of(p, m);
    s.theta = cplx(0.5 * (hi + lo), 0.0) - s.lam;
    s.delta = 0.5 * (hi - lo);
    s.a.assign(std::max(steps, 1), cplx(0));
    s.c.assign(std::max(steps, 1), cplx(0));
    s.a[0] = 0.0;
    s.c[0] = 1.0 / s.theta;
    const bool degenerate = s.delta <= 1e-300 || s.delta < 1e-15 * std::abs(s.theta);
    cplx rho = degenerate ? cplx(0) : s.delta / s.theta;
    for (int k = 1; k < steps; ++k) {
        if (degenerate) {
            s.a[k] = 0.0;
            s.c[k] = 0.0;
            continue;
        }
        const cplx rn = 1.0 / (2.0 * s.theta / s.delta - rho);
        s.a[k] = rn * rho;
        s.c[k] = 2.0 * rn / s.delta;
        rho = rn;
    }
    return s;
}

int validate_opts(const ac_problem* p, const ac_solve_opts* o, std::vector<int>& pm) {
    if (!o) return fail(AC_ERR_ARG, "opts is NULL");
    if (o->precision < 0 || o->precision > 2) return fail(AC_ERR_ARG, "unknown precision");
    if (o->inner != AC_INNER_CHEB && o->inner != AC_INNER_CHEB_CNN && o->inner != AC_INNER_CHEB_CNN_CYCLE &&
        o->inner != AC_INNER_CHEB_CNN_MR && o->inner != AC_INNER_EXACT && o->inner != AC_INNER_SP)
        return fail(AC_ERR_ARG, "unknown inner mode");
    pm.assign(p->ell, 0);
    if (o->inner == AC_INNER_SP) {
        if (!p->mgmem) return fail(AC_ERR_ARG, "no multigrid hierarchy (ac_problem_create_multigrid)");
        if (o->precision == AC_PREC_MIXED_BF16K)
            return fail(AC_ERR_UNSUPPORTED, "P_SP runs in float64 or float32 (AC_PREC_MIXED_FP32K)");
        for (int m = 0; m < p->ell; ++m) {
            const int v = o->p_per_shift ? o->p_per_shift[m] : o->p_uniform;
            if (v < 1 || v > 100000) return fail(AC_ERR_ARG, "inner iteration counts must be in [1, 100000]");
            if (m > 0 && v != pm[0]) return fail(AC_ERR_UNSUPPORTED, "P_SP runs the same iteration count for every shift");
            pm[m] = v;
        }
        return AC_OK;
    }
    if (o->inner == AC_INNER_EXACT) {
        if (p->g.periodic) return fail(AC_ERR_UNSUPPORTED, "the exact inner solve needs Dirichlet boundaries");
        if (p->kmin64 != p->kmax64) return fail(AC_ERR_UNSUPPORTED, "the exact inner solve needs a constant coefficient");
        return AC_OK;
    }
    if (o->inner != AC_INNER_CHEB && !p->cnn) return fail(AC_ERR_ARG, "no warm-start network attached");
    for (int m = 0; m < p->ell; ++m) {
        const int v = o->p_per_shift ? o->p_per_shift[m] : o->p_uniform;
        if (v < 1 || v > 100000) return fail(AC_ERR_ARG, "inner iteration counts must be in [1, 100000]");
        pm[m] = v;
    }
    for (int m = 1; m < p->ell; ++m)
        if (pm[m] != pm[p->ell - m]) return fail(AC_ERR_ARG, "conjugate shifts m and l-m need equal inner counts");
    return AC_OK;
}

// CNN inference buffers: inputs and two hidden activations (bf16, 16 channels) and the
// float32 output (2 channels).
size_t cnn_ws_bytes(const ac_problem* p) {
    const size_t px = static_cast<size_t>(p->ns) * static_cast<size_t>(p->g.n);
    return 3 * align_up(px * 32, 256) + align_up(px * 8, 256) + 256;
}

// exact inner solve: DST matrix, tridiagonal-scan carries
size_t exact_extra_bytes(const ac_problem* p, int prec) {
    return align_up(static_cast<size_t>(ac::dst_half_elems(p->g.nx)) * inner_elem(prec), 256) +
           align_up(ac::exact_carry_bytes(p->g.nx, p->g.ny, p->ns), 256);
}

size_t sp_extra_bytes(const ac_problem* p, int prec) {
    if (!p->mgmem) return 0;
    return ac::sp_ws_bytes(p->mg, p->g.n, p->nsc, p->nsr, prec != AC_PREC_FP64) + 256;
}

// Iterate buffers of the inner solve: four for the Chebyshev solves (x_q lives in
// buffer q mod 4, so that a sweep fusing two steps never writes a buffer another wave
// reads), two for the exact and saddle-point solves.
int iter_bufs(int inner) { return (inner == AC_INNER_EXACT || inner == AC_INNER_SP) ? 2 : 4; }

size_t prec_ws_bytes(const ac_problem* p, int prec, int inner) {
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    size_t b = (1 + iter_bufs(inner)) * align_up(static_cast<size_t>(off[p->ns]) * inner_elem(prec), 256) + 256;
    if (inner == AC_INNER_EXACT) b += exact_extra_bytes(p, prec);
    else if (inner == AC_INNER_SP) b += sp_extra_bytes(p, prec);
    else if (inner != AC_INNER_CHEB) b += cnn_ws_bytes(p);
    return b;
}


PrecBufs carve_prec(const ac_problem* p, int prec, void* ws, int inner) {
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    const size_t sz = align_up(static_cast<size_t>(off[p->ns]) * inner_elem(prec), 256);
    char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(ws), 256));
    const int nb = iter_bufs(inner);
    PrecBufs b{base, {base + sz, base + 2 * sz, nullptr, nullptr}, base + (1 + nb) * sz};
    if (nb == 4) {
        b.buf[2] = base + 3 * sz;
        b.buf[3] = base + 4 * sz;
    }
    return b;
}

// slot pointer into a spectral buffer
char* slot_ptr(const ac_problem* p, int prec, char* buf, int slot) {
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    return buf + off[slot_to_m(p, slot)] * inner_elem(prec);
}

void fill_twiddles(int ell, double* cw, double* sw) {
    for (int j = 0; j < ell; ++j) {
        cw[j] = std::cos(2.0 * kPi * j / ell);
        sw[j] = std::sin(2.0 * kPi * j / ell);
    }
}

// Arguments of the forward transform of r (scaled by in_scale) into the slots of rhat.
ac::FwdArgs fwd_args(ac_problem* p, int prec, const double* r, char* rhat, double in_scale) {
    ac::FwdArgs a{};
    a.n = p->g.n;
    for (int k = 0; k < p->ell; ++k) a.gam[k] = in_scale * std::pow(p->alpha, static_cast<double>(k) / p->ell);
    fill_twiddles(p->ell, a.cw, a.sw);
    a.r = r;
    for (int s = 0; s < p->ns; ++s) a.rhat[s] = slot_ptr(p, prec, rhat, s);
    return a;
}

int run_fwd(ac_problem* p, int prec, const double* r, char* rhat, double in_scale) {
    ac::FwdArgs a = fwd_args(p, prec, r, rhat, in_scale);
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    if (p->ctx->rec) {
        int vx, blocks;
        ac::fwd_geometry(a.n, vx, blocks);
        record_launch(p->ctx, ac::BOP_FWD, p->ell, prec, 0, vx, 4, blocks, a);
        return AC_OK;
    }
    const double bytes = 8.0 * p->ell * p->g.n + static_cast<double>(off[p->ns]) * inner_elem(prec);
    ProfScope ps(p->ctx, AC_K_TDFT_FWD, bytes);
    AC_HIP(ac::launch_tdft_fwd(p->ell, prec, a, p->ctx->stream));
    return AC_OK;
}

template <typename R>
void fill_cf(ac::ShiftCoef<R>& cf, int slot, const ChebShift& cs, int k) {
    cf.lam_re[slot] = static_cast<R>(cs.lam.real());
    cf.lam_im[slot] = static_cast<R>(cs.lam.imag());
    cf.a_re[slot] = static_cast<R>(cs.a[k].real());
    cf.a_im[slot] = static_cast<R>(cs.a[k].imag());
    cf.c_re[slot] = static_cast<R>(cs.c[k].real());
    cf.c_im[slot] = static_cast<R>(cs.c[k].imag());
    const cplx s = 1.0 / cs.theta;
    cf.s_re[slot] = static_cast<R>(s.real());
    cf.s_im[slot] = static_cast<R>(s.imag());
}

template <typename R>
void fill_coef(ac::SweepArgs<R>& a, int slot, const ChebShift& cs, int k) {
    fill_cf(a.cf, slot, cs, k);
}

// Bytes a sweep moves, per point, for one computing shift of element size esz.
double sweep_bytes_per_point(int curk, int prevk, bool final, double esz) {
    double n = 1.0;                                 // the stencil operand
    if (curk == ac::SRC_BUF) n += 1.0;              // rhat read separately
    if (prevk == ac::SRC_BUF) n += 1.0;             // x_{k-1}
    if (!final) n += 1.0;                           // x_{k+1} write
    return n * esz;
}

// Nested Chebyshev over all unique shifts.  warm: x_0 is in buf[0].  x_q lives in
// buf[q mod nb], nb = 4 when buf[2] and buf[3] are given (then runs of steady steps
// are fused in pairs), else 2.
// If z != nullptr the last sweep is fused with the inverse transform into z;
// otherwise the finished iterates are left in place and `where` reports them.
template <typename R>
int run_cheb_t(ac_problem* p, int prec, const std::vector<int>& pm, char* rhat, char* const buf[4], bool warm,
               double* z, std::vector<std::pair<int, char*>>* where, double out_scale) {
    const int ns = p->ns;
    int pmax = 0;
    std::vector<int> ps(ns);
    for (int s = 0; s < ns; ++s) {
        ps[s] = pm[slot_to_m(p, s)];
        pmax = std::max(pmax, ps[s]);
    }
    std::vector<ChebShift> cs(ns);
    for (int s = 0; s < ns; ++s) cs[s] = cheb_tables(p, prec, slot_to_m(p, s), pmax);

    const Tiling t = sweep_tiling(p);
    const double esz_c = 2.0 * sizeof(R), esz_r = sizeof(R);
    const double ksz = prec == AC_PREC_FP64 ? 8.0 : prec == AC_PREC_MIXED_BF16K ? 2.0 : 4.0;
    const void* kap = prec == AC_PREC_FP64 ? static_cast<const void*>(p->k64)
                      : prec == AC_PREC_MIXED_BF16K ? static_cast<const void*>(p->k16)
                                                    : static_cast<const void*>(p->k32);

    // first step index and the operand kinds for step k (computing x_{k+1})
    const int k_first = warm ? 0 : 1;
    auto kinds = [&](int k, int& curk, int& prevk) {
        if (warm) {
            curk = ac::SRC_BUF;
            prevk = (k == 0) ? ac::SRC_ZERO : ac::SRC_BUF;
        } else {
            curk = (k == 1) ? ac::SRC_RHAT : ac::SRC_BUF;
            prevk = (k == 1) ? ac::SRC_ZERO : (k == 2) ? ac::SRC_RHAT : ac::SRC_BUF;
        }
    };
    const int nb = (buf[2] && buf[3]) ? 4 : 2;
    // bq[q]: buffer holding x_q (-1: not stored).  A single step writes x_{k+1} over
    // x_{k-1} when that is in a buffer (each lane reads its points before writing them),
    // else into a buffer not holding x_k; a fused block writes its two outputs into the
    // two buffers it does not read (neighbouring waves read x_k and x_{k-1} on halos).
    std::vector<int> bq(static_cast<size_t>(std::max(pmax, 1)) + 4, -1);
    if (warm) bq[0] = 0;
    auto free_bufs = [&](int k, int* out, int want) {
        int got = 0;
        const int b0 = k >= 0 ? bq[k] : -1, b1 = k >= 1 ? bq[k - 1] : -1;
        for (int i = 0; i < nb && got < want; ++i)
            if (i != b0 && i != b1) out[got++] = i;
        return got == want;
    };
    auto single_out = [&](int k) {
        if (k >= 1 && bq[k - 1] >= 0) return bq[k - 1];
        int f[1];
        free_bufs(k, f, 1);
        return f[0];
    };
    // location of a finished iterate x_q
    auto fin_src = [&](int q, int& kind, int& bi) {
        if (!warm && q == 1) {
            kind = ac::SRC_RHAT;
            bi = -1;
        } else {
            kind = ac::SRC_BUF;
            bi = bq[q];
        }
    };

    const bool fuse = (z != nullptr);
    const int k_last = pmax - 1;  // step producing x_pmax
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    auto base_args = [&](ac::SweepArgs<R>& a) {
        a.g = p->g;
        a.t = t;
        a.kappa = kap;
        a.rhat = reinterpret_cast<const R*>(rhat);
        for (int i = 0; i < 4; ++i) a.bufs[i] = reinterpret_cast<const R*>(buf[i]);
        for (int s = 0; s < ns; ++s) a.soff[s] = static_cast<unsigned>(off[slot_to_m(p, s)]);
    };
    auto fill_final = [&](ac::SweepArgs<R>& a) {
        for (int kk = 0; kk < p->ell; ++kk)
            a.ginv[kk] = out_scale / (p->ell * std::pow(p->alpha, static_cast<double>(kk) / p->ell));
        fill_twiddles(p->ell, a.cw, a.sw);
        a.z = z;
    };
    int launched = 0;  // kernel launches of the current step (several with shift groups)
    // group g: real slot g (if any) and complex slots nsr + 2g, nsr + 2g + 1 (if any),
    // as slots 0, 1, 2 of the l = 5 variant; absent slots do not compute
    // (recording for a batch: always kMaxGroups records per step, empty ones with no
    // blocks, so that problems with different l record aligned sequences)
    auto launch_groups = [&](int curk, const ac::SweepArgs<R>& a, bool rec) -> hipError_t {
        const int ngroups = std::max(p->nsr, (p->nsc + 1) / 2);
        for (int grp = 0; grp < (rec ? kMaxGroups : ngroups); ++grp) {
            ac::SweepArgs<R> ga = a;
            const int map[3] = {grp < p->nsr ? grp : -1, 2 * grp < p->nsc ? p->nsr + 2 * grp : -1,
                                2 * grp + 1 < p->nsc ? p->nsr + 2 * grp + 1 : -1};
            bool anyc = false;
            for (int j = 0; j < 3; ++j) {
                const int sl = map[j];
                if (sl < 0) {
                    ga.src[j] = ac::SRC_BUF;
                    ga.soff[j] = 0;
                    continue;
                }
                ga.src[j] = a.src[sl];
                ga.fbuf[j] = a.fbuf[sl];
                ga.soff[j] = a.soff[sl];
                ga.cf.lam_re[j] = a.cf.lam_re[sl];
                ga.cf.lam_im[j] = a.cf.lam_im[sl];
                ga.cf.a_re[j] = a.cf.a_re[sl];
                ga.cf.a_im[j] = a.cf.a_im[sl];
                ga.cf.c_re[j] = a.cf.c_re[sl];
                ga.cf.c_im[j] = a.cf.c_im[sl];
                ga.cf.s_re[j] = a.cf.s_re[sl];
                ga.cf.s_im[j] = a.cf.s_im[sl];
                anyc = anyc || a.src[sl] == ac::SRC_COMPUTE;
            }
            if (rec) {
                record_launch(p->ctx, ac::BOP_STEP, 5, prec, curk, a.t.vx, a.t.wpb, anyc ? a.t.blocks : 0, ga);
                continue;
            }
            if (!anyc) continue;
            const hipError_t e = ac::launch_cheb_step(5, prec, curk, &ga, p->ctx->stream);
            if (e != hipSuccess) return e;
            ++launched;
        }
        return hipSuccess;
    };
    const bool groups = use_shift_groups(p);
    auto launch = [&](bool fin, int curk, const ac::SweepArgs<R>& a) -> hipError_t {
        launched = 1;
        if (p->ctx->rec) {
            if (!fin) return launch_groups(curk, a, true);
            record_launch(p->ctx, ac::BOP_FINAL, p->ell, prec, curk, a.t.vx, a.t.wpb, a.t.blocks, a);
            return hipSuccess;
        }
        if (fin) return ac::launch_cheb_final(p->ell, prec, curk, &a, p->ctx->stream);
        if (groups) {
            launched = 0;
            return launch_groups(curk, a, false);
        }
        return ac::launch_cheb_step(p->ell, prec, curk, &a, p->ctx->stream);
    };
    // Steady step k (x_k and x_{k-1} in buffers, not the fused last sweep).  Two
    // consecutive steady steps in which the same shifts compute run as one paired
    // sweep per shift group when four iterate buffers are available.
    // (the paired sweep addresses its buffers with 32-bit byte offsets below 2^31)
    const double spec_bytes = static_cast<double>(off[ns]) * sizeof(R);
    const bool fuse_ok = nb == 4 && p->ctx->pairs == 1 && !p->g.periodic && p->g.nx >= 3 &&
                         spec_bytes < 2147483648.0 && static_cast<double>(p->g.n) * ksz < 2147483648.0;
    const bool can_pair = fuse_ok;
    auto steady_step = [&](int k) {
        if (k > k_last || (fuse && k == k_last)) return false;
        int ck, pk;
        kinds(k, ck, pk);
        return ck == ac::SRC_BUF && pk == ac::SRC_BUF;
    };
    auto launch_pair = [&](int k, double& bytes) -> hipError_t {
        ac::PairArgs<R> pa{};
        pa.g = p->g;
        pa.t = pair_tiling(p, prec);
        pa.kappa = kap;
        pa.rhat = reinterpret_cast<const R*>(rhat);
        int f[2];
        if (!free_bufs(k, f, 2)) return hipErrorInvalidValue;
        bq[k + 1] = f[0];
        bq[k + 2] = f[1];
        pa.cur = reinterpret_cast<const R*>(buf[bq[k]]);
        pa.prev = reinterpret_cast<const R*>(buf[bq[k - 1]]);
        pa.out1 = reinterpret_cast<R*>(buf[bq[k + 1]]);
        pa.out2 = reinterpret_cast<R*>(buf[bq[k + 2]]);
        pa.bytes = static_cast<unsigned>(spec_bytes);
        bytes = 0.0;
        // recording for a batch: always kMaxGroups records, empty ones with no blocks
        const bool rec = p->ctx->rec != nullptr;
        const int ngroups = std::max(p->nsr, (p->nsc + 1) / 2);
        for (int grp = 0; grp < (rec ? kMaxGroups : ngroups); ++grp) {
            const int map[3] = {grp < p->nsr ? grp : -1, 2 * grp < p->nsc ? p->nsr + 2 * grp : -1,
                                2 * grp + 1 < p->nsc ? p->nsr + 2 * grp + 1 : -1};
            bool anyc = false;
            for (int j = 0; j < 3; ++j) {
                const int sl = map[j];
                pa.comp[j] = 0;
                pa.soff[j] = 0;
                if (sl < 0 || ps[sl] < k + 1) continue;
                pa.comp[j] = 1;
                pa.soff[j] = static_cast<unsigned>(off[slot_to_m(p, sl)]);
                fill_cf(pa.cf[0], j, cs[sl], k);
                fill_cf(pa.cf[1], j, cs[sl], k + 1);
                bytes += 5.0 * (slot_is_real(p, sl) ? esz_r : esz_c);  // x_k, x_{k-1}, rhat in; two out
                anyc = true;
            }
            if (rec) {
                record_launch(p->ctx, ac::BOP_PAIR, 2, prec, 0, pa.t.vx, pa.t.wpb, anyc ? pa.t.blocks : 0, pa);
                continue;
            }
            if (!anyc) continue;
            const hipError_t e = ac::launch_cheb_pair(prec, &pa, p->ctx->stream);
            if (e != hipSuccess) return e;
            ++launched;
        }
        // the pair's own minimum traffic: 5 vector streams per computing shift, kappa once
        // per launch (two unfused steps would move 8 streams and kappa twice)
        bytes = (bytes + static_cast<double>(launched) * ksz) * static_cast<double>(p->g.n);
        return hipSuccess;
    };
    // Three steps per sweep: one launch per block over every shift group (the real shifts
    // together, each complex shift alone), a workgroup per tile, a wave per group.
    // Recorded for a batch only with one budget for every shift, so that every problem
    // of the batch cuts its steps into the same blocks (aligned launch sequences).
    bool uniform = true;
    for (int s = 1; s < ns; ++s) uniform = uniform && ps[s] == ps[0];
    const bool can_triple = fuse_ok && p->ctx->triples == 1 && p->g.nx >= 4 && (!p->ctx->rec || uniform);
    // first: steps 1..3 from a zero guess (x_1 = rhat/theta and x_0 = 0 never stored)
    auto launch_triple = [&](int k, double& bytes, bool first) -> hipError_t {
        ac::TripleArgs<R> ta{};
        ta.g = p->g;
        ta.kappa = kap;
        ta.rhat = reinterpret_cast<const R*>(rhat);
        ta.first = first ? 1 : 0;
        int f[2];
        if (!free_bufs(k, f, 2)) return hipErrorInvalidValue;
        bq[k + 1] = -1;  // x_{k+1} stays in registers
        bq[k + 2] = f[0];
        bq[k + 3] = f[1];
        // (first: neither is read; any valid pointer)
        ta.cur = reinterpret_cast<const R*>(buf[first ? f[0] : bq[k]]);
        ta.prev = reinterpret_cast<const R*>(buf[first ? f[0] : bq[k - 1]]);
        ta.outz = reinterpret_cast<R*>(buf[bq[k + 2]]);
        ta.outw = reinterpret_cast<R*>(buf[bq[k + 3]]);
        ta.bytes = static_cast<unsigned>(spec_bytes);
        bytes = 0.0;
        auto add_group = [&](int kind, const int* slots, int count) {
            ac::TripleGroup<R> g{};
            g.kind = kind;
            bool anyc = false;
            for (int j = 0; j < 2; ++j) {
                const int sl = j < count ? slots[j] : -1;
                if (sl < 0 || ps[sl] < k + 1) continue;
                g.comp[j] = 1;
                g.soff[j] = static_cast<unsigned>(off[slot_to_m(p, sl)]);
                const ChebShift& c = cs[sl];
                const cplx sc = 1.0 / c.theta;  // x_1 = rhat / theta
                for (int t = 0; t < 3; ++t) {
                    const cplx at = c.a[k + t], ct = c.c[k + t];
                    cplx gt = 1.0 + at + ct * c.lam, ax = at, cx = ct;
                    if (first && t == 0) {
                        // x_2 from x_1 = s rhat, x_0 = 0, the window holding rhat:
                        // g x_1 + c (rhat - A' x_1) = (s g + c) rhat - (c s) A' rhat
                        gt = sc * gt + ct;
                        cx = ct * sc;
                        ax = 0.0;
                    } else if (first && t == 1) {
                        ax = at * sc;  // x_{k-1} = x_1 = s rhat, passed as rhat
                    }
                    g.g_re[t][j] = static_cast<R>(gt.real());
                    g.g_im[t][j] = static_cast<R>(gt.imag());
                    g.a_re[t][j] = static_cast<R>(ax.real());
                    g.a_im[t][j] = static_cast<R>(ax.imag());
                    g.c_re[t][j] = static_cast<R>(cx.real());
                    g.c_im[t][j] = static_cast<R>(cx.imag());
                }
                // the block's own minimum: x_k, x_{k-1}, rhat in, x_{k+2}, x_{k+3} out; from a
                // zero guess rhat in, two out
                bytes += (first ? 3.0 : 5.0) * (slot_is_real(p, sl) ? esz_r : esz_c);
                anyc = true;
            }
            if (anyc) ta.grp[ta.ngroups++] = g;
        };
        {
            const int sl[2] = {p->nsr > 0 ? 0 : -1, p->nsr > 1 ? 1 : -1};
            add_group(0, sl, 2);
        }
        for (int c = 0; c < p->nsc; ++c) {
            const int sl[1] = {p->nsr + c};
            add_group(1, sl, 1);
        }
        ta.t = triple_tiling(p, prec, std::max(ta.ngroups, 1));
        if (p->ctx->rec) {
            // batched: one record per block (its work list groups problems with equal group
            // counts; a problem with no computing shift records no blocks)
            record_launch(p->ctx, ac::BOP_TRIPLE, 3, prec, first ? 2 : 0, ta.t.vx, ta.t.wpb,
                          ta.ngroups > 0 ? ta.t.blocks : 0, ta);
            return hipSuccess;
        }
        if (ta.ngroups == 0) return hipSuccess;
        const hipError_t e = ac::launch_cheb_triple(prec, &ta, p->ctx->stream);
        if (e == hipSuccess) ++launched;
        // kappa once per launch (three unfused steps would move 12 vector streams per shift,
        // from a zero guess 9, and kappa three times)
        bytes = (bytes + static_cast<double>(launched) * ksz) * static_cast<double>(p->g.n);
        return e;
    };
    // length of the run of steady steps from k in which the same shifts compute
    auto steady_run = [&](int k) {
        int n = 0;
        while (steady_step(k + n)) {
            bool same = true;
            for (int s = 0; s < ns; ++s)
                if ((ps[s] >= k + 1) != (ps[s] >= k + n + 1)) same = false;
            if (!same) break;
            ++n;
        }
        return n;
    };
    // consecutive steady-state sweeps of one kind share one event pair
    std::unique_ptr<ProfScope> steady, paired, tripled;
    auto block_scope = [&](std::unique_ptr<ProfScope>& sc, int cls) {
        if (!sc) {
            sc = std::make_unique<ProfScope>(p->ctx, cls, 0.0);
            sc->launches = 0;
        }
    };
    for (int k = k_first; k <= k_last; ++k) {
        // the first three steps from a zero guess as one block, if the same shifts compute
        // in all three and none of them is the fused last sweep
        if (can_triple && !warm && k == 1 && 3 <= k_last && !(fuse && 3 == k_last)) {
            bool same = true;
            for (int s = 0; s < ns; ++s)
                if ((ps[s] >= 2) != (ps[s] >= 4)) same = false;
            if (same) {
                launched = 0;
                double bytes = 0.0;
                ProfScope ps_(p->ctx, AC_K_CHEB_FIRST, 0.0);
                AC_HIP(launch_triple(k, bytes, true));
                ps_.bytes = bytes;
                ps_.launches = launched;
                k += 2;  // x_4 done
                continue;
            }
        }
        // block size: greedy triples, then a pair or a single step (at 2048^2, l = 10 per
        // application: triple 211 us, pair 193 us, single 116 us, so a remainder of one
        // step is cheaper as a single than as two pairs replacing a triple)
        const int run = ((can_pair || can_triple) && steady_step(k)) ? steady_run(k) : 0;
        const int blk = (can_triple && run >= 3) ? 3 : (can_pair && run >= 2 ? 2 : 1);
        if (blk == 3) {
            steady.reset();
            paired.reset();
            block_scope(tripled, AC_K_CHEB_TRIPLE);
            launched = 0;
            double bytes = 0.0;
            AC_HIP(launch_triple(k, bytes, false));
            tripled->bytes += bytes;
            tripled->launches += launched;
            k += 2;  // x_{k+3} done
            continue;
        }
        if (blk == 2) {
            steady.reset();
            tripled.reset();
            block_scope(paired, AC_K_CHEB_PAIR);
            launched = 0;
            double bytes = 0.0;
            AC_HIP(launch_pair(k, bytes));
            paired->bytes += bytes;
            paired->launches += launched;
            ++k;  // x_{k+2} done
            continue;
        }
        paired.reset();
        tripled.reset();
        const bool final = fuse && (k == k_last);
        ac::SweepArgs<R> a{};
        base_args(a);
        int curk, prevk;
        kinds(k, curk, prevk);
        a.prevk = prevk;
        if (curk == ac::SRC_BUF && bq[k] < 0) return fail(AC_ERR_UNSUPPORTED, "internal: iterate x_k not stored");
        bq[k + 1] = single_out(k);
        a.cur = reinterpret_cast<const R*>(buf[bq[k] >= 0 ? bq[k] : 0]);
        a.out = reinterpret_cast<R*>(buf[bq[k + 1]]);
        a.prev = reinterpret_cast<const R*>(buf[k >= 1 && bq[k - 1] >= 0 ? bq[k - 1] : bq[k + 1]]);
        double bytes = 0.0;
        bool anyc = false;
        for (int s = 0; s < ns; ++s) {
            fill_coef(a, s, cs[s], k);
            const double esz = slot_is_real(p, s) ? esz_r : esz_c;
            if (ps[s] >= k + 1) {
                a.src[s] = ac::SRC_COMPUTE;
                anyc = true;
                bytes += sweep_bytes_per_point(curk, prevk, final, esz);
            } else {
                int kind, bi;
                fin_src(ps[s], kind, bi);
                a.src[s] = kind;
                a.fbuf[s] = bi < 0 ? 0 : bi;
                if (final) bytes += esz;
            }
        }
        if (anyc) bytes += ksz;
        bytes *= static_cast<double>(p->g.n);
        if (final) {
            bytes += 8.0 * p->ell * p->g.n;
            fill_final(a);
            ProfScope ps_(p->ctx, AC_K_CHEB_FINAL, bytes);
            AC_HIP(launch(true, curk, a));
        } else if (curk == ac::SRC_RHAT) {
            ProfScope ps_(p->ctx, AC_K_CHEB_FIRST, bytes);
            AC_HIP(launch(false, curk, a));
        } else {
            if (!steady) {
                steady = std::make_unique<ProfScope>(p->ctx, AC_K_CHEB_STEP, 0.0);
                steady->launches = 0;
            }
            steady->bytes += bytes;
            AC_HIP(launch(false, curk, a));
            steady->launches += launched;
        }
        if (steady && (k + 1 > k_last || (fuse && k + 1 == k_last))) steady.reset();
    }
    steady.reset();
    paired.reset();
    tripled.reset();
    if (fuse && k_last < k_first) {
        // nothing to iterate (cold start, every p = 1): x_1 = rhat/theta everywhere
        ac::SweepArgs<R> a{};
        base_args(a);
        a.prevk = ac::SRC_ZERO;
        double bytes = 0.0;
        for (int s = 0; s < ns; ++s) {
            fill_coef(a, s, cs[s], 0);
            a.src[s] = ac::SRC_RHAT;
            bytes += slot_is_real(p, s) ? esz_r : esz_c;
        }
        bytes = bytes * p->g.n + 8.0 * p->ell * p->g.n;
        fill_final(a);
        ProfScope ps_(p->ctx, AC_K_CHEB_FINAL, bytes);
        AC_HIP(launch(true, ac::SRC_BUF, a));
    }
    if (where) {
        where->clear();
        for (int s = 0; s < ns; ++s) {
            int kind, bi;
            fin_src(ps[s], kind, bi);
            where->emplace_back(kind, bi < 0 ? rhat : buf[bi]);
        }
    }
    return AC_OK;
}

int run_cheb(ac_problem* p, int prec, const std::vector<int>& pm, char* rhat, char* const buf[4], bool warm, double* z,
             std::vector<std::pair<int, char*>>* where, double out_scale) {
    if (prec == AC_PREC_FP64) return run_cheb_t<double>(p, prec, pm, rhat, buf, warm, z, where, out_scale);
    return run_cheb_t<float>(p, prec, pm, rhat, buf, warm, z, where, out_scale);
}

// Builds the per-slot arguments shared by the CNN input/output/residual kernels.
ac::CnnPrepArgs cnn_args(const ac_problem* p, int prec, const char* rhat) {
    ac::CnnPrepArgs a{};
    a.g = p->g;
    a.n = p->g.n;
    a.ns = p->ns;
    a.rhat = rhat;
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    for (int s = 0; s < p->ns; ++s) {
        const int m = slot_to_m(p, s);
        a.soff[s] = static_cast<unsigned>(off[m]);
        a.is_real[s] = slot_is_real(p, s) ? 1 : 0;
        const cplx lam = shift_of(p, m);
        a.lam_re[s] = static_cast<float>(lam.real());
        a.lam_im[s] = static_cast<float>(lam.imag());
        a.inv_scale[s] = 1.f;
        a.scale[s] = 1.f;
        a.fac_re[s] = 1.f;
        a.fac_im[s] = 0.f;
    }
    a.kappa = p->k64;
    a.c0 = p->cnn ? p->cnn->c0 : 0.0;
    a.c1 = p->cnn ? p->cnn->c1 : 1.0;
    return a;
}


int slot_residuals(ac_problem* p, int prec, const ac::CnnPrepArgs& a, const char* x0, SlotStats& out) {
    const void* kap = prec == AC_PREC_FP64 ? static_cast<const void*>(p->k64)
                      : prec == AC_PREC_MIXED_BF16K ? static_cast<const void*>(p->k16)
                                                    : static_cast<const void*>(p->k32);
    AC_HIP(ac::launch_cnn_resid(prec, a, x0, kap, p->rpart, kResidBlocks, p->ctx->stream));
    std::vector<double> h(static_cast<size_t>(kResidBlocks) * 4 * kMaxShift);
    AC_HIP(hipMemcpyAsync(h.data(), p->rpart, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->ctx->stream));
    AC_HIP(hipStreamSynchronize(p->ctx->stream));
    out.rr.assign(p->ns, 0.0);
    out.bb.assign(p->ns, 0.0);
    out.cr.assign(p->ns, 0.0);
    out.ci.assign(p->ns, 0.0);
    for (int b = 0; b < kResidBlocks; ++b)
        for (int s = 0; s < p->ns; ++s) {
            const double* q = &h[static_cast<size_t>(b) * 4 * kMaxShift + 4 * s];
            out.rr[s] += q[0];
            out.bb[s] += q[1];
            out.cr[s] += q[2];
            out.ci[s] += q[3];
        }
    return AC_OK;
}

// Input scales s_m = RMS(rhat_m) into the argument block (and optionally to the host).
void set_rms_scales(const ac_problem* p, const SlotStats& st, ac::CnnPrepArgs& a, double* scales) {
    for (int s = 0; s < p->ns; ++s) {
        const double rms = std::sqrt(st.rr[s] / static_cast<double>(p->g.n));
        a.scale[s] = static_cast<float>(rms);
        a.inv_scale[s] = rms > 0 ? static_cast<float>(1.0 / rms) : 0.f;
        if (scales) scales[s] = rms;
    }
}

int cnn_forward_impl(ac_cnn* c, const uint16_t* x, int B, int H, int W, float* y, uint16_t* a1, uint16_t* a2,
                     hipStream_t st) {
    ac::CnnConvArgs ca{};
    ca.B = B;
    ca.H = H;
    ca.W = W;
    ca.in = x;
    ca.w = c->wf;
    ca.bias = c->bias;
    ca.relu = 1;
    ca.out16 = a1;
    AC_HIP(ac::launch_cnn_conv(ca, st));
    ca.in = a1;
    ca.w = c->wf + 2304;
    ca.bias = c->bias + 16;
    ca.out16 = a2;
    AC_HIP(ac::launch_cnn_conv(ca, st));
    ca.in = a2;
    ca.w = c->wf + 2 * 2304;
    ca.bias = c->bias + 32;
    ca.relu = 0;
    ca.out16 = nullptr;
    ca.out32 = y;
    ca.nout = 2;
    AC_HIP(ac::launch_cnn_conv(ca, st));
    return AC_OK;
}

// In-place complex scaling of one spectral slot (n points, interleaved if complex).
template <typename R>
__global__ void slot_scale_kernel(R* x, long long n, int cplx_, R sr, R si) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cplx_) {
        const R a = x[2 * i], b = x[2 * i + 1];
        x[2 * i] = sr * a - si * b;
        x[2 * i + 1] = sr * b + si * a;
    } else {
        x[i] = sr * x[i];
    }
}

// Learned initial guesses for every shift slot, written into x0buf.  With scaling on
// each slot's output is multiplied by the complex factor c that minimises
// |rhat - c B x0| (a one-dimensional minimal-residual step).  A slot whose (scaled)
// guess leaves a residual of at least accept * |rhat|, or is not finite, is reset to
// zero.
int cnn_warm_start(ac_problem* p, int prec, const char* rhat, char* x0buf, char* cws, int* fallbacks) {
    const size_t px = static_cast<size_t>(p->ns) * static_cast<size_t>(p->g.n);
    uint16_t* X = reinterpret_cast<uint16_t*>(cws);
    uint16_t* A1 = reinterpret_cast<uint16_t*>(cws + align_up(px * 32, 256));
    uint16_t* A2 = reinterpret_cast<uint16_t*>(cws + 2 * align_up(px * 32, 256));
    float* Y = reinterpret_cast<float*>(cws + 3 * align_up(px * 32, 256));
    ac::CnnPrepArgs a = cnn_args(p, prec, rhat);
    SlotStats st;
    {
        ProfScope ps(p->ctx, AC_K_CNN, 0.0);
        AC_TRY(slot_residuals(p, prec, a, nullptr, st));
    }
    set_rms_scales(p, st, a, nullptr);
    a.x = X;
    const bool fused = p->cnn->fused != 0;
    if (fused) {
        long long off[kMaxShift + 1];
        spectral_offsets(p, off);
        const double bytes = 2.0 * static_cast<double>(off[p->ns]) * inner_elem(prec) + 8.0 * p->g.n;
        ProfScope ps(p->ctx, AC_K_CNN, bytes);
        AC_HIP(ac::launch_cnn_fused(prec, a, p->cnn->wf, p->cnn->bias, x0buf, p->ctx->stream));
    } else {
        const double bytes = static_cast<double>(px) * (32.0 * 7 + 8.0 * 2) + 8.0 * p->g.n;
        ProfScope ps(p->ctx, AC_K_CNN, bytes);
        AC_HIP(ac::launch_cnn_prep(prec, a, p->ctx->stream));
        AC_TRY(cnn_forward_impl(p->cnn, X, p->ns, p->g.ny, p->g.nx, Y, A1, A2, p->ctx->stream));
        AC_HIP(ac::launch_cnn_post(prec, a, Y, x0buf, p->ctx->stream));
    }
    {
        ProfScope ps(p->ctx, AC_K_CNN, 0.0);
        AC_TRY(slot_residuals(p, prec, a, x0buf, st));
    }
    std::vector<int> reject(p->ns, 0);
    bool rescale = false;
    for (int s = 0; s < p->ns; ++s) {
        double c_re = 1.0, c_im = 0.0;
        if (p->cnn->scaled && st.bb[s] > 0.0) {
            c_re = st.cr[s] / st.bb[s];
            c_im = st.ci[s] / st.bb[s];
        }
        const double res = st.res(s, c_re, c_im);
        const double bound = p->cnn->accept * p->cnn->accept * st.rr[s];
        reject[s] = !(std::isfinite(res) && std::isfinite(c_re) && std::isfinite(c_im) && res < bound);
        a.fac_re[s] = static_cast<float>(c_re);
        a.fac_im[s] = static_cast<float>(c_im);
        rescale = rescale || (!reject[s] && (c_re != 1.0 || c_im != 0.0));
    }
    if (rescale && !fused) {
        ProfScope ps(p->ctx, AC_K_CNN, static_cast<double>(px) * 16.0);
        AC_HIP(ac::launch_cnn_post(prec, a, Y, x0buf, p->ctx->stream));
    } else if (rescale) {
        // the fused kernel wrote scale * y: multiply by the factor in place
        ProfScope ps(p->ctx, AC_K_CNN, static_cast<double>(px) * 16.0);
        const int blocks = static_cast<int>((p->g.n + 255) / 256);
        for (int s = 0; s < p->ns; ++s) {
            if (reject[s] || (a.fac_re[s] == 1.f && a.fac_im[s] == 0.f)) continue;
            char* base = slot_ptr(p, prec, x0buf, s);
            const int cx = slot_is_real(p, s) ? 0 : 1;
            if (prec == AC_PREC_FP64)
                hipLaunchKernelGGL((slot_scale_kernel<double>), dim3(blocks), dim3(256), 0, p->ctx->stream,
                                   reinterpret_cast<double*>(base), p->g.n, cx, static_cast<double>(a.fac_re[s]),
                                   static_cast<double>(a.fac_im[s]));
            else
                hipLaunchKernelGGL((slot_scale_kernel<float>), dim3(blocks), dim3(256), 0, p->ctx->stream,
                                   reinterpret_cast<float*>(base), p->g.n, cx, a.fac_re[s], a.fac_im[s]);
            AC_HIP(hipGetLastError());
        }
    }
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    for (int s = 0; s < p->ns; ++s) {
        if (!reject[s]) continue;
        const int m = slot_to_m(p, s);
        AC_HIP(ac::launch_zero_bytes(x0buf, off[m] * static_cast<long long>(inner_elem(prec)),
                                     slice_elems(p, m) * static_cast<long long>(inner_elem(prec)), p->ctx->stream));
        if (fallbacks) ++*fallbacks;
    }
    return AC_OK;
}

ac::InvArgs inv_args(const ac_problem* p, int prec, char* yhat, double* z) {
    ac::InvArgs a{};
    a.n = p->g.n;
    for (int k = 0; k < p->ell; ++k) a.ginv[k] = 1.0 / (p->ell * std::pow(p->alpha, static_cast<double>(k) / p->ell));
    fill_twiddles(p->ell, a.cw, a.sw);
    for (int s = 0; s < p->ns; ++s) a.yhat[s] = slot_ptr(p, prec, yhat, s);
    a.z = z;
    return a;
}

// Exact shifted solves (A - lambda_m I) yhat_m = rhat_m for a constant coefficient,
// then the inverse time-DFT into z.  The slots are split into planes P (one per real
// slot, two per complex slot) with the even/odd butterfly along x, transformed by the
// two half sine matrices (one GEMM each over all planes), solved along y into P,
// transformed back by the transposed halves and merged into the rhat slots with the
// inverse butterfly.
int exact_inner(ac_problem* p, int prec, const PrecBufs& b, double* z) {
    ac_ctx* c = p->ctx;
    hipStream_t st = c->stream;
    const int nx = p->g.nx, ny = p->g.ny;
    char* P = b.buf[0];
    char* T = b.buf[1];
    char* S = b.cnn;
    char* carry = S + align_up(static_cast<size_t>(ac::dst_half_elems(nx)) * inner_elem(prec), 256);
    ac::ExactArgs a{};
    a.n = p->g.n;
    a.nx = nx;
    a.ny = ny;
    a.dim = p->g.dim;
    a.nslot = p->ns;
    a.kappa = p->kmin64;
    int planes = 0;
    for (int s = 0; s < p->ns; ++s) {
        const cplx lam = shift_of(p, slot_to_m(p, s));
        a.slot[s] = slot_ptr(p, prec, b.rhat, s);
        a.cplx[s] = slot_is_real(p, s) ? 0 : 1;
        a.plane[s] = planes;
        // the real slots' shifts are real; drop the rounding residue of the polar form
        a.lr[s] = lam.real();
        a.li[s] = a.cplx[s] ? lam.imag() : 0.0;
        planes += a.cplx[s] ? 2 : 1;
    }
    const double esz = static_cast<double>(inner_elem(prec));
    const double pn = static_cast<double>(planes) * p->g.n;
    const int h = (nx + 1) / 2, h2 = nx / 2;
    // split/merge 4 pn, two GEMM operand passes 4 pn + the half matrices twice,
    // tridiagonal scan 6 pn, inverse DFT
    const double bytes = esz * (14.0 * pn + 2.0 * ac::dst_half_elems(nx)) + 8.0 * p->ell * p->g.n +
                         esz * static_cast<double>(p->nsr + 2 * p->nsc) * p->g.n;
    ProfScope ps(c, AC_K_EXACT, bytes);
    AC_HIP(ac::launch_dst_half(prec, S, nx, st));
    AC_HIP(ac::launch_exact_planes(prec, true, a, P, st));
    const long long cols = static_cast<long long>(ny) * planes;
    if (cols > 2147483647LL) return fail(AC_ERR_UNSUPPORTED, "too many plane columns for the sine transform");
    // Cm[off.., :] = op(half) * Bm[off.., :]; even block rows [0, h), odd block rows [h, nx)
    auto gemm = [&](bool inverse, const char* Bm, char* Cm) -> int {
        const size_t esz_b = inner_elem(prec);
        for (int half = 0; half < 2; ++half) {
            const int d = half == 0 ? h : h2;
            if (d == 0) continue;
            const size_t moff = half == 0 ? 0 : static_cast<size_t>(h) * h;  // matrix entries
            const size_t roff = half == 0 ? 0 : static_cast<size_t>(h);      // block row
            AC_HIP(ac::launch_sine_gemm(prec == AC_PREC_FP64 ? 0 : 1, inverse, S + moff * esz_b, d,
                                        Bm + roff * esz_b, nx, Cm + roff * esz_b, nx, static_cast<int>(cols), st));
        }
        return AC_OK;
    };
    AC_TRY(gemm(false, P, T));
    AC_HIP(ac::launch_exact_tridiag(prec, a, T, P, carry, st));
    AC_TRY(gemm(true, P, T));
    AC_HIP(ac::launch_exact_planes(prec, false, a, T, st));
    AC_HIP(ac::launch_tdft_inv(p->ell, prec, inv_args(p, prec, b.rhat, z), st));
    return AC_OK;
}

// P_SP: every shifted solve by saddle-point MINRES (complex shifts) or CG (real shifts)
// with multigrid preconditioners, pm[0] iterations each, then the inverse time-DFT; in
// float32 (vectors and multigrid coefficients) for AC_PREC_MIXED_FP32K.
int sp_inner(ac_problem* p, int prec, int iters, const PrecBufs& b, double* z) {
    ac::SpProblem P{};
    P.h = &p->mg;
    P.n = p->g.n;
    for (int s = 0; s < p->ns; ++s) {
        const cplx lam = shift_of(p, slot_to_m(p, s));
        char* in = slot_ptr(p, prec, b.rhat, s);
        char* out = slot_ptr(p, prec, b.buf[0], s);
        if (slot_is_real(p, s)) {
            P.lam[P.nr] = lam.real();
            P.br[P.nr] = in;
            P.yr[P.nr++] = out;
        } else {
            P.sigma[P.nc] = std::abs(lam.imag());
            P.rho[P.nc] = lam.real();
            P.im_pos[P.nc] = lam.imag() > 0.0 ? 1 : 0;
            P.bc[P.nc] = in;
            P.yc[P.nc++] = out;
        }
    }
    char* ws = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(b.cnn), 256));
    // per iteration: the saddle / CG operators (2 resp. 1 products with A), a V-cycle per
    // vector, the Lanczos / CG vector updates and two inner products
    const double ne = static_cast<double>(inner_elem(prec)) * p->g.n;
    const double bytes = iters * ne * (p->nsc * 2.0 * 12.0 + p->nsr * 10.0);
    ProfScope ps(p->ctx, AC_K_SADDLE, bytes);
    ac_ctx* c = p->ctx;
    if (!c->graphs) {
        AC_HIP(ac::sp_solve(P, iters, prec != AC_PREC_FP64, ws, c->stream));
    } else {
        // Every argument of the inner solve is fixed by the problem, the workspace, the
        // step count and the precision, so one capture serves every later application.
        ac_problem::SpGraph& gr = p->spg;
        if (!(gr.exec && gr.ws == ws && gr.iters == iters && gr.prec == prec)) {
            if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
            gr = ac_problem::SpGraph{};
            AC_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
            const hipError_t le = ac::sp_solve(P, iters, prec != AC_PREC_FP64, ws, c->cap);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(c->cap, &graph);
            if (le != hipSuccess || ee != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(AC_ERR_HIP, std::string("P_SP graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ee));
            }
            const hipError_t ie = hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                gr.exec = nullptr;
                return fail(AC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
            }
            gr.ws = ws;
            gr.iters = iters;
            gr.prec = prec;
        }
        AC_HIP(hipGraphLaunch(gr.exec, c->stream));
    }
    AC_HIP(ac::launch_tdft_inv(p->ell, prec, inv_args(p, prec, b.buf[0], z), p->ctx->stream));
    return AC_OK;
}

int apply_prec_impl(ac_problem* p, const ac_solve_opts* o, const std::vector<int>& pm, const double* r, double* z,
                    void* ws, double in_scale, int* fallbacks) {
    const PrecBufs b = carve_prec(p, o->precision, ws, o->inner);
    AC_TRY(run_fwd(p, o->precision, r, b.rhat, in_scale));
    if (o->inner == AC_INNER_SP) {
        AC_TRY(sp_inner(p, o->precision, pm[0], b, z));
    } else if (o->inner == AC_INNER_EXACT) {
        AC_TRY(exact_inner(p, o->precision, b, z));
    } else if (o->inner != AC_INNER_CHEB) {
        AC_TRY(cnn_warm_start(p, o->precision, b.rhat, b.buf[0], b.cnn, fallbacks));
        AC_TRY(run_cheb(p, o->precision, pm, b.rhat, b.buf, true, z, nullptr));
    } else {
        AC_TRY(run_cheb(p, o->precision, pm, b.rhat, b.buf, false, z, nullptr));
    }
    return AC_OK;
}

bool prec_from_rhat_ok(const ac_problem* p, const ac_solve_opts* o) {
    (void)p;
    return o->inner == AC_INNER_CHEB || o->inner == AC_INNER_CHEB_CNN_CYCLE || o->inner == AC_INNER_CHEB_CNN_MR;
}

int axpy_fwd_impl(ac_problem* p, const ac_solve_opts* o, const ac::VecSet& vs, int nv, double* w, void* ws,
                  double* partial, int stride, int* blocks) {
    if (p->ctx->rec) return fail(AC_ERR_UNSUPPORTED, "the fused Gram-Schmidt update is not batched");
    const PrecBufs b = carve_prec(p, o->precision, ws, o->inner);
    ac::AxpyFwdArgs a{};
    a.f = fwd_args(p, o->precision, nullptr, b.rhat, 1.0);
    for (int q = 0; q < nv; ++q) {
        a.v[q] = vs.v[q];
        a.c[q] = vs.s2[q];
    }
    a.nv = nv;
    a.stride = stride;
    a.w = w;
    a.partial = partial;
    *blocks = ac::axpy_fwd_blocks(p->g.n);
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    const double len = static_cast<double>(p->ell) * p->g.n;
    ProfScope ps(p->ctx, AC_K_KRYLOV, 8.0 * len * (nv + 2) + static_cast<double>(off[p->ns]) * inner_elem(o->precision));
    AC_HIP(ac::launch_axpy_fwd(p->ell, o->precision, a, p->ctx->stream));
    return AC_OK;
}

int apply_prec_rhat(ac_problem* p, const ac_solve_opts* o, const std::vector<int>& pm, double* z, void* ws,
                    double out_scale) {
    const PrecBufs b = carve_prec(p, o->precision, ws, o->inner);
    return run_cheb(p, o->precision, pm, b.rhat, b.buf, false, z, nullptr, out_scale);
}

int calA_impl(ac_problem* p, const double* x, double* y, const double* b, double* partial) {
    ac::CalAArgs a{};
    a.g = p->g;
    a.t = calA_tiling(p);
    a.kappa = p->k64;
    a.x = x;
    a.y = y;
    a.b = b;
    a.partial = partial;
    a.ell = p->ell;
    if (p->kblocks) a.kappa = p->kblocks;
    if (p->ctx->rec) {
        if (p->kblocks) return fail(AC_ERR_UNSUPPORTED, "varying diagonal blocks are not batched");
        // curk carries the form (strips or halo loads), which a batched launch must share
        record_launch(p->ctx, b ? ac::BOP_CALA_RES : ac::BOP_CALA, p->ell, 0, ac::calA_strips(p->g) ? 1 : 0, a.t.vx,
                      a.t.wpb, a.t.blocks, a);
        return AC_OK;
    }
    const double kbytes = p->kblocks ? 8.0 * p->ell * p->g.n : 8.0 * p->g.n;
    const double bytes = (b ? 24.0 : 16.0) * p->ell * p->g.n + kbytes;
    ProfScope ps(p->ctx, AC_K_APPLY_CALA, bytes);
    if (p->kblocks) AC_HIP(ac::launch_apply_calA_var(p->ell, b != nullptr, a, p->ctx->stream));
    else AC_HIP(ac::launch_apply_calA(p->ell, b != nullptr, a, p->ctx->stream));
    return AC_OK;
}

long long calA_partials(const ac_problem* p) { return calA_tiling(p).tiles * (p->kblocks ? p->ell : 1); }

}  // namespace ach

// ---------------------------------------------------------------------------
// ABI (every definition below matches an extern "C" declaration of alphacirc.h)

const char* ac_status_string(int s) {
    switch (s) {
        case AC_OK: return "ok";
        case AC_NOT_CONVERGED: return "not converged";
        case AC_ERR_ARG: return "invalid argument";
        case AC_ERR_ALPHA: return "alpha outside (0, mu_lo^l)";
        case AC_ERR_BOUNDS: return "invalid spectral bounds";
        case AC_ERR_HIP: return "HIP runtime error";
        case AC_ERR_WORKSPACE: return "workspace too small";
        case AC_ERR_NONFINITE: return "non-finite or non-positive value";
        case AC_ERR_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* ac_last_error(void) { return g_last_error.c_str(); }

int ac_ctx_create(int device, void* stream, ac_ctx** out) {
    if (!out) return fail(AC_ERR_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    AC_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(AC_ERR_ARG, "device index out of range");
    AC_HIP(hipSetDevice(device));
    auto* c = new ac_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->pinned), kPinnedDoubles * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return fail(AC_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipHostFree(c->pinned);
        delete c;
        return fail(AC_ERR_HIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
    }
    const int ns = ac::noalloc_scratch_init(device);
    if (ns < 0) {
        (void)hipStreamDestroy(c->cap);
        (void)hipHostFree(c->pinned);
        delete c;
        return ns;
    }
    *out = c;
    return AC_OK;
}

int ac_ctx_destroy(ac_ctx* c) {
    if (!c) return AC_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto& p : c->pool) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return AC_OK;
}

int ac_ctx_set_graphs(ac_ctx* c, int on) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    c->graphs = on != 0;
    return AC_OK;
}

int ac_ctx_set_stream(ac_ctx* c, void* stream) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    c->stream = static_cast<hipStream_t>(stream);
    return AC_OK;
}

int ac_ctx_set_profiling(ac_ctx* c, int on) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    c->profiling = on != 0;
    return AC_OK;
}

int ac_ctx_kernel_stats(ac_ctx* c, double* ms, long long* launches, double* bytes) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    AC_TRY(harvest(c));
    for (int i = 0; i < AC_K_COUNT; ++i) {
        if (ms) ms[i] = c->ms[i];
        if (launches) launches[i] = c->launches[i];
        if (bytes) bytes[i] = c->bytes[i];
    }
    return AC_OK;
}

int ac_ctx_reset_stats(ac_ctx* c) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    AC_TRY(harvest(c));
    for (int i = 0; i < AC_K_COUNT; ++i) {
        c->ms[i] = 0;
        c->launches[i] = 0;
        c->bytes[i] = 0;
    }
    return AC_OK;
}

int ac_problem_create(ac_ctx* c, const ac_grid* grid, const double* kappa, int ell, double alpha,
                      const ac_bounds* bounds, ac_problem** out) {
    if (!out) return fail(AC_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!c || !grid || !kappa) return fail(AC_ERR_ARG, "NULL argument");
    if (grid->dim != 1 && grid->dim != 2) return fail(AC_ERR_ARG, "dim must be 1 or 2");
    if (grid->nx < 1 || grid->ny < 1) return fail(AC_ERR_ARG, "grid sizes must be positive");
    if (grid->dim == 1 && grid->ny != 1) return fail(AC_ERR_ARG, "dim 1 needs ny == 1");
    if (grid->bc != AC_BC_DIRICHLET && grid->bc != AC_BC_PERIODIC) return fail(AC_ERR_ARG, "unknown boundary");
    if (ell < 2 || ell > kMaxEll) return fail(AC_ERR_UNSUPPORTED, "l must be in [2, 16]");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(AC_ERR_ALPHA, "alpha must be positive and finite");
    if (static_cast<long long>(grid->nx) * grid->ny > (1LL << 31) - 1) return fail(AC_ERR_UNSUPPORTED, "N too large");
    if (block_elems_too_large(static_cast<long long>(grid->nx) * grid->ny, ell))
        return fail(AC_ERR_UNSUPPORTED, "l*N too large (block vectors use 32-bit element offsets)");
    AC_HIP(hipSetDevice(c->device));

    auto* p = new ac_problem();
    p->ctx = c;
    p->g.nx = grid->nx;
    p->g.ny = grid->ny;
    p->g.dim = grid->dim;
    p->g.periodic = grid->bc == AC_BC_PERIODIC;
    p->g.n = static_cast<long long>(grid->nx) * grid->ny;
    p->ell = ell;
    p->alpha = alpha;
    p->nsr = (ell % 2 == 0) ? 2 : 1;
    p->nsc = (ell - p->nsr) / 2;
    p->ns = p->nsr + p->nsc;
    const size_t n = static_cast<size_t>(p->g.n);
    const int nblk = ac::setup_blocks();
    double* partial = nullptr;
    auto cleanup = [&]() {
        if (p->k64) (void)hipFree(p->k64);
        if (p->k32) (void)hipFree(p->k32);
        if (p->k16) (void)hipFree(p->k16);
        if (p->rpart) (void)hipFree(p->rpart);
        if (partial) (void)hipFree(partial);
        delete p;
    };
    hipError_t e = hipMalloc(&p->k64, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->k32, align_up(n * sizeof(float), 256));
    if (e == hipSuccess) e = hipMalloc(&p->k16, align_up(n * sizeof(uint16_t), 256));
    if (e == hipSuccess) e = hipMalloc(&p->rpart, static_cast<size_t>(kResidBlocks) * 4 * kMaxShift * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&partial, nblk * 8 * sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(p->k64, kappa, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = ac::launch_kappa_setup(p->g, p->k64, p->k32, p->k16, partial, nblk, c->stream);
    std::vector<double> h(nblk * 8);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), partial, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        cleanup();
        return fail(AC_ERR_HIP, std::string("problem set-up: ") + hipGetErrorString(e));
    }
    (void)hipFree(partial);
    partial = nullptr;
    // 0 min kappa, 1 max Gershgorin (float64), 2/3 the same in float32, 4/5 in bf16,
    // 6 count of invalid kappa, 7 max kappa
    double q[8] = {1e308, 0, 1e308, 0, 1e308, 0, 0, 0};
    for (int b = 0; b < nblk; ++b) {
        for (int i = 0; i < 6; ++i) q[i] = (i % 2 == 0) ? std::min(q[i], h[b * 8 + i]) : std::max(q[i], h[b * 8 + i]);
        q[6] += h[b * 8 + 6];
        q[7] = std::max(q[7], h[b * 8 + 7]);
    }
    if (q[6] != 0.0 || !(q[0] > 0.0)) {
        cleanup();
        return fail(AC_ERR_NONFINITE, "kappa must be finite and positive everywhere");
    }
    // lambda_min of the integer -Delta_h stencil (Dirichlet), 0 for periodic
    double lmin = 0.0;
    if (!p->g.periodic) {
        lmin = 4.0 * std::pow(std::sin(kPi / (2.0 * (p->g.nx + 1))), 2);
        if (p->g.dim == 2) lmin += 4.0 * std::pow(std::sin(kPi / (2.0 * (p->g.ny + 1))), 2);
    }
    p->kmin64 = q[0];
    p->kmax64 = q[7];
    if (bounds) {
        if (!(bounds->mu_lo >= 1.0 - 1e-12) || !(bounds->mu_hi >= bounds->mu_lo) || !std::isfinite(bounds->mu_hi)) {
            cleanup();
            return fail(AC_ERR_BOUNDS, "need 1 <= mu_lo <= mu_hi < inf");
        }
        for (int i = 0; i < 3; ++i) {
            p->bounds[i][0] = bounds->mu_lo;
            p->bounds[i][1] = bounds->mu_hi;
        }
    } else {
        p->bounds[AC_PREC_FP64][0] = 1.0 + q[0] * lmin;
        p->bounds[AC_PREC_FP64][1] = q[1];
        p->bounds[AC_PREC_MIXED_FP32K][0] = 1.0 + q[2] * lmin;
        p->bounds[AC_PREC_MIXED_FP32K][1] = q[3];
        p->bounds[AC_PREC_MIXED_BF16K][0] = 1.0 + q[4] * lmin;
        p->bounds[AC_PREC_MIXED_BF16K][1] = q[5];
    }
    // Corollary 1 / Lemma 1: 0 < alpha < mu_lo^l (alpha != mu_j^l for all j)
    const double mulo = std::min({p->bounds[0][0], p->bounds[1][0], p->bounds[2][0]});
    if (!(alpha < std::pow(mulo, ell))) {
        cleanup();
        return fail(AC_ERR_ALPHA, "alpha must satisfy 0 < alpha < mu_lo^l");
    }
    *out = p;
    return AC_OK;
}

int ac_problem_create_blocks(ac_ctx* c, const ac_grid* grid, const double* kappa_blocks, int ell, double alpha,
                             const ac_bounds* bounds, ac_problem** out) {
    if (!out) return fail(AC_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!c || !grid || !kappa_blocks) return fail(AC_ERR_ARG, "NULL argument");
    if (ell < 2 || ell > kMaxEll) return fail(AC_ERR_UNSUPPORTED, "l must be in [2, 16]");
    if (grid->nx < 1 || grid->ny < 1) return fail(AC_ERR_ARG, "grid sizes must be positive");
    if (static_cast<long long>(grid->nx) * grid->ny > (1LL << 31) - 1) return fail(AC_ERR_UNSUPPORTED, "N too large");
    if (block_elems_too_large(static_cast<long long>(grid->nx) * grid->ny, ell))
        return fail(AC_ERR_UNSUPPORTED, "l*N too large (block vectors use 32-bit element offsets)");
    AC_HIP(hipSetDevice(c->device));
    const size_t n = static_cast<size_t>(grid->nx) * static_cast<size_t>(grid->ny);
    const int nblk = ac::setup_blocks();
    double* mean = nullptr;
    double* bad = nullptr;
    double* kb = nullptr;
    auto cleanup = [&]() {
        if (mean) (void)hipFree(mean);
        if (bad) (void)hipFree(bad);
        if (kb) (void)hipFree(kb);
    };
    hipError_t e = hipMalloc(&mean, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&bad, nblk * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&kb, static_cast<size_t>(ell) * n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(kb, kappa_blocks, static_cast<size_t>(ell) * n * sizeof(double),
                                            hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = ac::launch_kappa_mean(kb, ell, static_cast<long long>(n), mean, bad, c->stream);
    std::vector<double> h(nblk);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), bad, nblk * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        cleanup();
        return fail(AC_ERR_HIP, std::string("block coefficients: ") + hipGetErrorString(e));
    }
    double nbad = 0.0;
    for (double v : h) nbad += v;
    if (nbad != 0.0) {
        cleanup();
        return fail(AC_ERR_NONFINITE, "every block's kappa must be finite and positive");
    }
    // the representative block A(mean kappa) defines the preconditioner and its bounds
    ac_problem* p = nullptr;
    const int st = ac_problem_create(c, grid, mean, ell, alpha, bounds, &p);
    (void)hipFree(mean);
    mean = nullptr;
    (void)hipFree(bad);
    bad = nullptr;
    if (st < 0) {
        cleanup();
        return st;
    }
    p->kblocks = kb;
    *out = p;
    return AC_OK;
}

int ac_problem_destroy(ac_problem* p) {
    if (!p) return AC_OK;
    (void)hipSetDevice(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    (void)hipFree(p->k64);
    (void)hipFree(p->k32);
    (void)hipFree(p->k16);
    (void)hipFree(p->rpart);
    if (p->kblocks) (void)hipFree(p->kblocks);
    if (p->mgmem) (void)hipFree(p->mgmem);
    if (p->spg.exec) (void)hipGraphExecDestroy(p->spg.exec);
    delete p;
    return AC_OK;
}

int ac_problem_create_multigrid(ac_problem* p) {
    if (!p) return fail(AC_ERR_ARG, "problem is NULL");
    if (p->mgmem) return AC_OK;
    if (p->g.periodic) return fail(AC_ERR_UNSUPPORTED, "the multigrid hierarchy needs Dirichlet boundaries");
    if (p->g.n >= (1LL << 31)) return fail(AC_ERR_UNSUPPORTED, "the multigrid kernels index points with 32 bits");
    ac::MgHierarchy h{};
    h.nlev = ac::mg_plan(p->g.dim, p->g.nx, p->g.ny, h.lev);
    if (h.nlev < 1) return fail(AC_ERR_UNSUPPORTED, "grid too large for the multigrid hierarchy");
    size_t total = 0;
    for (int l = 0; l < h.nlev; ++l) total += align_up(ac::mg_level_doubles(h.lev[l]), 32);
    AC_HIP(hipSetDevice(p->ctx->device));
    double* mem = nullptr;
    AC_HIP(hipMalloc(reinterpret_cast<void**>(&mem), total * sizeof(double)));
    double* q = mem;
    for (int l = 0; l < h.nlev; ++l) {
        ac::MgLevel& L = h.lev[l];
        double* b = q;
        L.diag = b;
        L.wx = b + L.n;
        L.wy = b + 2 * L.n;
        L.bx0 = b + 3 * L.n;
        L.bx1 = L.bx0 + L.ny;
        L.by0 = L.bx1 + L.ny;
        L.by1 = L.by0 + L.nx;
        L.diag_f = reinterpret_cast<float*>(L.by1 + L.nx);
        L.wx_f = L.diag_f + L.n;
        L.wy_f = L.wx_f + L.n;
        q += align_up(ac::mg_level_doubles(L), 32);
    }
    hipError_t e = ac::mg_build(h, p->k64, p->ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return fail(AC_ERR_HIP, std::string("multigrid set-up: ") + hipGetErrorString(e));
    }
    p->mg = h;
    p->mgmem = mem;
    return AC_OK;
}

int ac_mg_workspace_size(const ac_problem* p, int nvec, size_t* bytes) {
    if (!p || !bytes) return fail(AC_ERR_ARG, "NULL argument");
    if (!p->mgmem) return fail(AC_ERR_ARG, "no multigrid hierarchy (ac_problem_create_multigrid)");
    if (nvec < 1 || nvec > ac::kMgMaxVec) return fail(AC_ERR_ARG, "nvec out of range");
    *bytes = ac::mg_scratch_elems(p->mg, nvec) * sizeof(double) + 256;
    return AC_OK;
}

int ac_mg_vcycle(ac_problem* p, int nvec, const double* shifts, const double* b, double* u, void* ws, size_t ws_bytes) {
    if (!p || !shifts || !b || !u) return fail(AC_ERR_ARG, "NULL argument");
    if (!p->mgmem) return fail(AC_ERR_ARG, "no multigrid hierarchy (ac_problem_create_multigrid)");
    if (nvec < 1 || nvec > ac::kMgMaxVec) return fail(AC_ERR_ARG, "nvec out of range");
    for (int q = 0; q < nvec; ++q)
        if (!(shifts[q] < p->bounds[AC_PREC_FP64][0])) return fail(AC_ERR_ARG, "every shift must be below mu_lo");
    if (!ws || ws_bytes < ac::mg_scratch_elems(p->mg, nvec) * sizeof(double) + 256)
        return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(p->ctx->device));
    const double* bs[ac::kMgMaxVec];
    double* us[ac::kMgMaxVec];
    for (int q = 0; q < nvec; ++q) {
        bs[q] = b + static_cast<size_t>(q) * p->g.n;
        us[q] = u + static_cast<size_t>(q) * p->g.n;
    }
    double* scratch = reinterpret_cast<double*>(align_up(reinterpret_cast<size_t>(ws), 256));
    AC_HIP(ac::mg_vcycle(p->mg, nvec, bs, us, shifts, scratch, p->ctx->stream));
    return AC_OK;
}

int ac_spectral_bounds(const ac_problem* p, double* lo, double* hi) {
    if (!p) return fail(AC_ERR_ARG, "problem is NULL");
    if (lo) *lo = p->bounds[AC_PREC_FP64][0];
    if (hi) *hi = p->bounds[AC_PREC_FP64][1];
    return AC_OK;
}

int ac_problem_dims(const ac_problem* p, long long* n, int* ell, int* ns) {
    if (!p) return fail(AC_ERR_ARG, "problem is NULL");
    if (n) *n = p->g.n;
    if (ell) *ell = p->ell;
    if (ns) *ns = p->ns;
    return AC_OK;
}

int ac_problem_shifts(const ac_problem* p, double* lam) {
    if (!p || !lam) return fail(AC_ERR_ARG, "NULL argument");
    for (int m = 0; m < p->ell; ++m) {
        const cplx l = shift_of(p, m);
        lam[2 * m] = l.real();
        lam[2 * m + 1] = l.imag();
    }
    return AC_OK;
}

int ac_alloc_nc2(const ac_problem* p, double budget, int* out) {
    if (!p || !out) return fail(AC_ERR_ARG, "NULL argument");
    if (!(budget > 0)) return fail(AC_ERR_ARG, "budget must be positive");
    const double lo = p->bounds[AC_PREC_FP64][0], hi = p->bounds[AC_PREC_FP64][1];
    std::vector<double> r(p->ell);
    double sum = 0.0;
    auto sigma = [&](double re) {
        const double k = (hi - re) / (lo - re);
        return (std::sqrt(k) - 1.0) / (std::sqrt(k) + 1.0);
    };
    const double a1 = std::pow(p->alpha, 1.0 / p->ell);
    const double s0 = sigma(a1);
    for (int m = 0; m < p->ell; ++m) {
        const double re = a1 * std::cos(2.0 * kPi * m / p->ell);
        r[m] = std::log(s0) / std::log(sigma(re));
        sum += r[m];
    }
    for (int m = 0; m < p->ell; ++m) out[m] = std::max(1, static_cast<int>(std::floor(r[m] / sum * budget)));
    return AC_OK;
}

int ac_alloc_nc1(const ac_problem* p, double budget, int* out) {
    if (!p || !out) return fail(AC_ERR_ARG, "NULL argument");
    if (!(budget > 0)) return fail(AC_ERR_ARG, "budget must be positive");
    const int v = std::max(1, static_cast<int>(std::floor(budget / p->ell)));
    for (int m = 0; m < p->ell; ++m) out[m] = v;
    return AC_OK;
}

int ac_prec_workspace_size(const ac_problem* p, const ac_solve_opts* o, size_t* bytes) {
    if (!p || !o || !bytes) return fail(AC_ERR_ARG, "NULL argument");
    if (o->precision < 0 || o->precision > 2) return fail(AC_ERR_ARG, "unknown precision");
    *bytes = prec_ws_bytes(p, o->precision, o->inner);
    return AC_OK;
}

namespace ach {
size_t vec_bytes(const ac_problem* p) { return align_up(static_cast<size_t>(p->ell) * p->g.n * sizeof(double), 256); }
size_t solve_ws_bytes(const ac_problem* p, const ac_solve_opts* o) {
    const int m = o->restart_m;
    size_t b = 256;
    b += static_cast<size_t>(2 * m + 1) * vec_bytes(p);
    b += align_up(static_cast<size_t>(ac::krylov_blocks()) * 72 * sizeof(double), 256);
    b += align_up(static_cast<size_t>(calA_partials(p)) * sizeof(double), 256);
    b += align_up(128 * sizeof(double), 256);
    b += prec_ws_bytes(p, o->precision, o->inner);
    return b;
}
SolveWs carve_solve(const ac_problem* p, const ac_solve_opts* o, void* ws) {
    SolveWs w{};
    char* b = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(ws), 256));
    const size_t vb = vec_bytes(p);
    for (int i = 0; i <= o->restart_m; ++i, b += vb) w.V[i] = reinterpret_cast<double*>(b);
    for (int i = 0; i < o->restart_m; ++i, b += vb) w.Z[i] = reinterpret_cast<double*>(b);
    w.partial = reinterpret_cast<double*>(b);
    b += align_up(static_cast<size_t>(ac::krylov_blocks()) * 72 * sizeof(double), 256);
    w.partial2 = reinterpret_cast<double*>(b);
    b += align_up(static_cast<size_t>(calA_partials(p)) * sizeof(double), 256);
    w.red = reinterpret_cast<double*>(b);
    b += align_up(128 * sizeof(double), 256);
    w.prec = b;
    return w;
}
}  // namespace ach

int ac_solve_workspace_size(const ac_problem* p, const ac_solve_opts* o, size_t* bytes) {
    if (!p || !o || !bytes) return fail(AC_ERR_ARG, "NULL argument");
    if (o->restart_m < 1 || o->restart_m > 32) return fail(AC_ERR_UNSUPPORTED, "restart_m must be in [1, 32]");
    if (o->precision < 0 || o->precision > 2) return fail(AC_ERR_ARG, "unknown precision");
    *bytes = solve_ws_bytes(p, o);
    return AC_OK;
}

int ac_apply_A(ac_problem* p, const double* x, double* y) {
    if (!p || !x || !y) return fail(AC_ERR_ARG, "NULL argument");
    if (ranges_overlap(x, y, block_bytes(p))) return fail(AC_ERR_ARG, "x and y overlap");
    AC_HIP(hipSetDevice(p->ctx->device));
    return calA_impl(p, x, y, nullptr, nullptr);
}

int ac_apply_prec(ac_problem* p, const ac_solve_opts* o, const double* r, double* z, void* ws, size_t ws_bytes) {
    if (!p || !r || !z) return fail(AC_ERR_ARG, "NULL argument");
    if (ranges_overlap(r, z, block_bytes(p))) return fail(AC_ERR_ARG, "r and z overlap");
    std::vector<int> pm;
    AC_TRY(validate_opts(p, o, pm));
    if (!ws || ws_bytes < prec_ws_bytes(p, o->precision, o->inner)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(p->ctx->device));
    return apply_prec_impl(p, o, pm, r, z, ws, 1.0);
}

int ac_spectral_offsets(const ac_problem* p, int prec, long long* offsets) {
    if (!p || !offsets) return fail(AC_ERR_ARG, "NULL argument");
    if (prec < 0 || prec > 2) return fail(AC_ERR_ARG, "unknown precision");
    spectral_offsets(p, offsets);
    return AC_OK;
}

int ac_tdft_forward(ac_problem* p, int prec, const double* r, void* rhat) {
    if (!p || !r || !rhat) return fail(AC_ERR_ARG, "NULL argument");
    if (prec < 0 || prec > 2) return fail(AC_ERR_ARG, "unknown precision");
    AC_HIP(hipSetDevice(p->ctx->device));
    return run_fwd(p, prec, r, static_cast<char*>(rhat), 1.0);
}

namespace ach {
__global__ void zero_kernel(double* x, long long n) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

__global__ void zero_kernel_int(int* x, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = 0;
}

hipError_t launch_zero(double* x, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_zero_int(int* x, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_kernel_int, dim3(1), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

template <typename R>
__global__ void scale_copy_kernel(R* dst, const R* src, long long n, int cplx_, R sr, R si) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cplx_) {
        const R a = src[2 * i], b = src[2 * i + 1];
        dst[2 * i] = sr * a - si * b;
        dst[2 * i + 1] = sr * b + si * a;
    } else {
        dst[i] = sr * src[i];
    }
}

template <typename R>
int gather_t(ac_problem* p, int prec, const std::vector<std::pair<int, char*>>& where, char* rhat, char* yhat) {
    const int blocks = static_cast<int>((p->g.n + 255) / 256);
    for (int s = 0; s < p->ns; ++s) {
        const int m = slot_to_m(p, s);
        const ChebShift cs = cheb_tables(p, prec, m, 1);
        const cplx sc = where[s].first == ac::SRC_RHAT ? 1.0 / cs.theta : cplx(1.0);
        R* dst = reinterpret_cast<R*>(slot_ptr(p, prec, yhat, s));
        const R* src = reinterpret_cast<const R*>(slot_ptr(p, prec, where[s].second, s));
        hipLaunchKernelGGL((scale_copy_kernel<R>), dim3(blocks), dim3(256), 0, p->ctx->stream, dst, src, p->g.n,
                           slot_is_real(p, s) ? 0 : 1, static_cast<R>(sc.real()), static_cast<R>(sc.imag()));
        AC_HIP(hipGetLastError());
    }
    (void)rhat;
    return AC_OK;
}
}  // namespace ach

int ac_shifted_cheb(ac_problem* p, const ac_solve_opts* o, const void* rhat, const void* x0hat, void* yhat, void* ws,
                    size_t ws_bytes) {
    if (!p || !rhat || !yhat) return fail(AC_ERR_ARG, "NULL argument");
    std::vector<int> pm;
    AC_TRY(validate_opts(p, o, pm));
    if (o->inner == AC_INNER_EXACT || o->inner == AC_INNER_SP)
        return fail(AC_ERR_UNSUPPORTED, "ac_shifted_cheb runs the Chebyshev solves");
    if (!ws || ws_bytes < prec_ws_bytes(p, o->precision)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(p->ctx->device));
    const int prec = o->precision;
    PrecBufs b = carve_prec(p, prec, ws);
    long long off[kMaxShift + 1];
    spectral_offsets(p, off);
    const size_t sbytes = static_cast<size_t>(off[p->ns]) * inner_elem(prec);
    AC_HIP(hipMemcpyAsync(b.rhat, rhat, sbytes, hipMemcpyDeviceToDevice, p->ctx->stream));
    const bool warm = x0hat != nullptr;
    if (warm) AC_HIP(hipMemcpyAsync(b.buf[0], x0hat, sbytes, hipMemcpyDeviceToDevice, p->ctx->stream));
    std::vector<std::pair<int, char*>> where;
    AC_TRY(run_cheb(p, prec, pm, b.rhat, b.buf, warm, nullptr, &where));
    if (prec == AC_PREC_FP64) return gather_t<double>(p, prec, where, b.rhat, static_cast<char*>(yhat));
    return gather_t<float>(p, prec, where, b.rhat, static_cast<char*>(yhat));
}

int ac_tdft_inverse(ac_problem* p, int prec, const void* yhat, double* z) {
    if (!p || !yhat || !z) return fail(AC_ERR_ARG, "NULL argument");
    if (prec < 0 || prec > 2) return fail(AC_ERR_ARG, "unknown precision");
    AC_HIP(hipSetDevice(p->ctx->device));
    const ac::InvArgs a = inv_args(p, prec, const_cast<char*>(static_cast<const char*>(yhat)), z);
    AC_HIP(ac::launch_tdft_inv(p->ell, prec, a, p->ctx->stream));
    return AC_OK;
}

