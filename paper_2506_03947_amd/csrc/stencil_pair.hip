// Two steady shifted-Chebyshev steps in one marching sweep (temporal blocking).
//
// A steady step of the three-term recurrence (Section 3) reads x_k (stencil),
// x_{k-1} and rhat and writes x_{k+1}: four vector streams per shift and step.  Fusing
// steps k and k+1 reads x_k, x_{k-1}, rhat and writes x_{k+1}, x_{k+2}: five streams
// per two steps.  x_{k+1} is never re-read from memory: the wave keeps a three-row
// window of it in registers and recomputes it on a one-row / one-column halo of its
// tile (the halo rows of x_k, kappa, x_{k-1} and rhat are shared with the
// neighbouring chunks through L2).
//
// Mapping.  A wave owns a strip of 64*VX computed columns and a chunk of h rows.
// Strips advance by 64*VX - 2 columns: the first and last column of a strip are
// computed for x_{k+1} only (their outer neighbour is not), and the x_{k+2} values of
// the 64*VX - 2 inner columns are the strip's output (plus column 0 in the first
// strip, whose outer neighbour is the Dirichlet ghost).  Every point of the grid is
// written by exactly one wave.  Dirichlet grids only.
//
// Arithmetic per point is the single-step sweep's, term for term, so the iterates
// agree with two single steps up to rounding (the compiler may contract the same
// expressions differently in another kernel: a few ulps).
#include "stencil_kernels.h"

namespace ac {
namespace {

template <typename R, typename KS, int VX>
__device__ __forceinline__ void cheb_pair_body(const PairArgs<R>& a, int bid, int nb) {
    using K = R;
    constexpr int NC = 2;             // complex slots 1, 2
    constexpr int W = kWave * VX;     // computed columns per strip

    // the tile is uniform across the wave: scalar registers for everything derived from
    // it, scalar branches for the row tests
    const int tile = __builtin_amdgcn_readfirstlane(static_cast<int>(tile_of_wave(a.t, bid, nb)));
    if (tile < 0) return;
    const int nx = a.g.nx, ny = a.g.ny;
    const int lane = threadIdx.x & (kWave - 1);
    const int sx = static_cast<int>(tile % a.t.nsx);
    const int cy = static_cast<int>(tile / a.t.nsx);
    const int x0 = sx * (W - 2);
    const int y0 = cy * a.t.h;
    const int y1 = min(y0 + a.t.h, ny);
    const KS* __restrict__ kap = static_cast<const KS*>(a.kappa);

    const bool cr = a.comp[0] != 0;
    bool cc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) cc[c] = a.comp[1 + c] != 0;

    const int xb = x0 + lane * VX;
    const bool lane_ok = xb < nx;  // VX = 2 only on even nx: a lane is wholly in or out
    const bool hl = (lane == 0 || lane == kWave - 1);
    const int hx = (lane == 0) ? x0 - 1 : x0 + W;
    const bool hok = hl && hx >= 0 && hx < nx;
    // columns whose x_{k+2} this wave writes (and x_{k+1}, on its own rows)
    bool own[VX];
    bool own_all = true, own_any = false;
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int c = xb + v;
        own[v] = lane_ok && (c >= x0 + 1 || c == 0) && c <= x0 + W - 2;
        own_all = own_all && own[v];
        own_any = own_any || own[v];
    }

    // x_k and kappa (storage type): three-row windows (with the strip-edge halo values)
    KS kw[3][VX], kh[3];
    R xr[3][VX], xrh[3];
    R xc[3][NC][2 * VX], xch[3][NC][2];
    // x_{k+1}: three-row window (no halo: the strip-edge columns are not owned)
    R yr[3][VX];
    R yc[3][NC][2 * VX];
    KS kprev[VX];                      // kappa of the row below the x_{k+2} row
    R hr0[VX], hc0[NC][2 * VX];        // rhat, row of the x_{k+2} update
    R hr1[VX], hc1[NC][2 * VX];        // rhat, row of the x_{k+1} update
    R pr[VX], pc[NC][2 * VX];          // x_{k-1}, row of the x_{k+1} update

    // Buffer loads over byte ranges: lanes past the grid edge, lanes that fetch no halo
    // value and halo values outside the grid read zeros (the Dirichlet ghosts) with no
    // lane-divergent branch, so the loads of a row all stay in flight together.
    const unsigned nR = static_cast<unsigned>(sizeof(R));
    const __amdgpu_buffer_rsrc_t rk = buf_rsrc(kap, static_cast<unsigned>(a.g.n) * sizeof(KS));
    const __amdgpu_buffer_rsrc_t rx = buf_rsrc(a.cur, a.bytes);
    const __amdgpu_buffer_rsrc_t rp = buf_rsrc(a.prev, a.bytes);
    const __amdgpu_buffer_rsrc_t rh = buf_rsrc(a.rhat, a.bytes);

    auto load_row = [&](auto S_, int y) {
        constexpr int S = decltype(S_)::value;
#pragma unroll
        for (int v = 0; v < VX; ++v) kw[S][v] = KS(0), xr[S][v] = R(0);
        kh[S] = KS(0);
        xrh[S] = R(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int v = 0; v < 2 * VX; ++v) xc[S][c][v] = R(0);
            xch[S][c][0] = xch[S][c][1] = R(0);
        }
        if (y < 0 || y >= ny) return;  // Dirichlet ghost row (uniform)
        const unsigned rowp = static_cast<unsigned>(y) * static_cast<unsigned>(nx);
        const unsigned pt = rowp + static_cast<unsigned>(xb);
        const unsigned hp = rowp + static_cast<unsigned>(hx);
        bld<0>(rk, lane_ok ? pt * static_cast<unsigned>(sizeof(KS)) : kOob, kw[S]);
        {
            KS t[1];
            bld<0>(rk, hok ? hp * static_cast<unsigned>(sizeof(KS)) : kOob, t);
            kh[S] = t[0];
        }
        if (cr) {
            const unsigned o = a.soff[0];
            bld<0>(rx, lane_ok ? (o + pt) * nR : kOob, xr[S]);
            R t[1];
            bld<0>(rx, hok ? (o + hp) * nR : kOob, t);
            xrh[S] = t[0];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (cc[c]) {
                const unsigned o = a.soff[1 + c];
                bld<0>(rx, lane_ok ? (o + 2u * pt) * nR : kOob, xc[S][c]);
                bld<0>(rx, hok ? (o + 2u * hp) * nR : kOob, xch[S][c]);
            }
        }
    };

    // rhat and x_{k-1} of row y (for the x_{k+1} update).  The chunk's halo rows are
    // also read by the neighbouring chunk: plain loads there, non-temporal inside.
    // Lanes past the grid edge read zeros (their x_{k+1} is zeroed anyway).
    auto load_centre = [&](int y) {
#pragma unroll
        for (int v = 0; v < VX; ++v) hr1[v] = pr[v] = R(0);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int v = 0; v < 2 * VX; ++v) hc1[c][v] = pc[c][v] = R(0);
        if (y < 0 || y >= ny) return;
        const unsigned pt = static_cast<unsigned>(y) * static_cast<unsigned>(nx) + static_cast<unsigned>(xb);
        const bool inner = (y >= y0 && y < y1);
        if (cr) {
            const unsigned off = lane_ok ? (a.soff[0] + pt) * nR : kOob;
            if (inner) {
                bld<2>(rh, off, hr1);
                bld<2>(rp, off, pr);
            } else {
                bld<0>(rh, off, hr1);
                bld<0>(rp, off, pr);
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (cc[c]) {
                const unsigned off = lane_ok ? (a.soff[1 + c] + 2u * pt) * nR : kOob;
                if (inner) {
                    bld<2>(rh, off, hc1[c]);
                    bld<2>(rp, off, pc[c]);
                } else {
                    bld<0>(rh, off, hc1[c]);
                    bld<0>(rp, off, pc[c]);
                }
            }
        }
    };

    // face coefficients of row y: kappa row y (slot C, with the halo), its south and
    // north rows' centre values
    auto row_faces = [&](Faces<K> (&fc)[VX], const KS (&kr)[VX], KS khr, const KS (&ks)[VX], const KS (&kn)[VX],
                         int y) {
        K kc[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) kc[v] = kconv(kr[v]);
        const K khc = kconv(khr);
        const K kwv = shfl_up1(kc[VX - 1]);
        const K kev = shfl_dn1(kc[0]);
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const K kwest = (v > 0) ? kc[v - 1] : (lane == 0 ? khc : kwv);
            const K keast = (v < VX - 1) ? kc[v + 1] : (lane == kWave - 1 ? khc : kev);
            fc[v] = faces<K>(a.g, xb + v, y, kc[v], kwest, keast, kconv(ks[v]), kconv(kn[v]));
        }
    };

    auto store_row = [&](R* base, unsigned off, int y, auto N_, const R* vals) {
        constexpr int N = decltype(N_)::value;  // values per point (1 real, 2 complex)
        if (!own_any) return;
        const unsigned pt = static_cast<unsigned>(y) * static_cast<unsigned>(nx) + static_cast<unsigned>(xb);
        R* d = base + off + static_cast<unsigned>(N) * pt;
        if (own_all) {
            R t[N * VX];
#pragma unroll
            for (int i = 0; i < N * VX; ++i) t[i] = vals[i];
            stv_nt<R, N * VX>(d, t);
        } else {
            // strip-edge lanes: the owned points one by one (N values each)
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                if (own[v]) {
                    R t[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) t[i] = vals[N * v + i];
                    stv<R, N>(d + N * v, t);
                }
            }
        }
    };

    // x_{k+1} of row y from the x_k / kappa window slots (P, C, N) = rows (y-1, y, y+1),
    // into x_{k+1} slot Y; stored when y is one of the chunk's rows.
    auto step1 = [&](auto P_, auto C_, auto N_, auto Y_, int y) {
        constexpr int P = decltype(P_)::value, C = decltype(C_)::value, N = decltype(N_)::value;
        constexpr int Y = decltype(Y_)::value;
        const ShiftCoef<R>& cf = a.cf[0];
        const bool live = (y >= 0 && y < ny);  // uniform
        Faces<K> fc[VX];
        row_faces(fc, kw[C], kh[C], kw[P], kw[N], y);
        const bool st = live && y >= y0 && y < y1;
        if (cr) {
            const R wv = shfl_up1(xr[C][VX - 1]);
            const R ev = shfl_dn1(xr[C][0]);
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R uw = (v > 0) ? xr[C][v - 1] : (lane == 0 ? xrh[C] : wv);
                const R ue = (v < VX - 1) ? xr[C][v + 1] : (lane == kWave - 1 ? xrh[C] : ev);
                const R uc = xr[C][v];
                R bu = (fc[v].diag - cf.lam_re[0]) * uc;
                bu -= fc[v].w * uw + fc[v].e * ue + fc[v].s * xr[P][v] + fc[v].n * xr[N][v];
                const R nv = uc + cf.a_re[0] * (uc - pr[v]) + cf.c_re[0] * (hr1[v] - bu);
                yr[Y][v] = (live && lane_ok) ? nv : R(0);
            }
            if (st) store_row(a.out1, a.soff[0], y, std::integral_constant<int, 1>{}, yr[Y]);
        } else {
#pragma unroll
            for (int v = 0; v < VX; ++v) yr[Y][v] = R(0);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int s = 1 + c;
            if (cc[c]) {
                const R wre = shfl_up1(xc[C][c][2 * VX - 2]);
                const R wim = shfl_up1(xc[C][c][2 * VX - 1]);
                const R ere = shfl_dn1(xc[C][c][0]);
                const R eim = shfl_dn1(xc[C][c][1]);
                const R hre = xch[C][c][0], him = xch[C][c][1];
                const R lr = cf.lam_re[s], li = cf.lam_im[s];
                const R ar = cf.a_re[s], ai = cf.a_im[s];
                const R kr = cf.c_re[s], ki = cf.c_im[s];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const R uwr = (v > 0) ? xc[C][c][2 * v - 2] : (lane == 0 ? hre : wre);
                    const R uwi = (v > 0) ? xc[C][c][2 * v - 1] : (lane == 0 ? him : wim);
                    const R uer = (v < VX - 1) ? xc[C][c][2 * v + 2] : (lane == kWave - 1 ? hre : ere);
                    const R uei = (v < VX - 1) ? xc[C][c][2 * v + 3] : (lane == kWave - 1 ? him : eim);
                    const R ucr = xc[C][c][2 * v], uci = xc[C][c][2 * v + 1];
                    const R dl = fc[v].diag - lr;
                    R bur = dl * ucr + li * uci;
                    R bui = dl * uci - li * ucr;
                    bur -= fc[v].w * uwr + fc[v].e * uer + fc[v].s * xc[P][c][2 * v] + fc[v].n * xc[N][c][2 * v];
                    bui -= fc[v].w * uwi + fc[v].e * uei + fc[v].s * xc[P][c][2 * v + 1] +
                           fc[v].n * xc[N][c][2 * v + 1];
                    const R dr = ucr - pc[c][2 * v], di = uci - pc[c][2 * v + 1];
                    const R qr = hc1[c][2 * v] - bur, qi = hc1[c][2 * v + 1] - bui;
                    const R nr = ucr + (ar * dr - ai * di) + (kr * qr - ki * qi);
                    const R ni = uci + (ar * di + ai * dr) + (kr * qi + ki * qr);
                    yc[Y][c][2 * v] = (live && lane_ok) ? nr : R(0);
                    yc[Y][c][2 * v + 1] = (live && lane_ok) ? ni : R(0);
                }
                if (st) store_row(a.out1, a.soff[s], y, std::integral_constant<int, 2>{}, yc[Y][c]);
            } else {
#pragma unroll
                for (int v = 0; v < 2 * VX; ++v) yc[Y][c][v] = R(0);
            }
        }
    };

    // x_{k+2} of row y (one of the chunk's rows) from the x_{k+1} slots (P, C, N) =
    // rows (y-1, y, y+1); x_k of row y is x_k / kappa slot KC, kappa of row y+1 slot KN.
    auto step2 = [&](auto P_, auto C_, auto N_, auto KC_, auto KN_, int y) {
        constexpr int P = decltype(P_)::value, C = decltype(C_)::value, N = decltype(N_)::value;
        constexpr int KC = decltype(KC_)::value, KN = decltype(KN_)::value;
        const ShiftCoef<R>& cf = a.cf[1];
        Faces<K> fc[VX];
        row_faces(fc, kw[KC], kh[KC], kprev, kw[KN], y);
        if (cr) {
            const R wv = shfl_up1(yr[C][VX - 1]);
            const R ev = shfl_dn1(yr[C][0]);
            R z[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                // the strip-edge neighbours are not computed: zero, which is exact at a
                // Dirichlet edge and only reaches columns this wave does not write otherwise
                const R uw = (v > 0) ? yr[C][v - 1] : (lane == 0 ? R(0) : wv);
                const R ue = (v < VX - 1) ? yr[C][v + 1] : (lane == kWave - 1 ? R(0) : ev);
                const R uc = yr[C][v];
                R bu = (fc[v].diag - cf.lam_re[0]) * uc;
                bu -= fc[v].w * uw + fc[v].e * ue + fc[v].s * yr[P][v] + fc[v].n * yr[N][v];
                z[v] = uc + cf.a_re[0] * (uc - xr[KC][v]) + cf.c_re[0] * (hr0[v] - bu);
            }
            store_row(a.out2, a.soff[0], y, std::integral_constant<int, 1>{}, z);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int s = 1 + c;
            if (cc[c]) {
                const R wre = shfl_up1(yc[C][c][2 * VX - 2]);
                const R wim = shfl_up1(yc[C][c][2 * VX - 1]);
                const R ere = shfl_dn1(yc[C][c][0]);
                const R eim = shfl_dn1(yc[C][c][1]);
                const R lr = cf.lam_re[s], li = cf.lam_im[s];
                const R ar = cf.a_re[s], ai = cf.a_im[s];
                const R kr = cf.c_re[s], ki = cf.c_im[s];
                R z[2 * VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const R uwr = (v > 0) ? yc[C][c][2 * v - 2] : (lane == 0 ? R(0) : wre);
                    const R uwi = (v > 0) ? yc[C][c][2 * v - 1] : (lane == 0 ? R(0) : wim);
                    const R uer = (v < VX - 1) ? yc[C][c][2 * v + 2] : (lane == kWave - 1 ? R(0) : ere);
                    const R uei = (v < VX - 1) ? yc[C][c][2 * v + 3] : (lane == kWave - 1 ? R(0) : eim);
                    const R ucr = yc[C][c][2 * v], uci = yc[C][c][2 * v + 1];
                    const R dl = fc[v].diag - lr;
                    R bur = dl * ucr + li * uci;
                    R bui = dl * uci - li * ucr;
                    bur -= fc[v].w * uwr + fc[v].e * uer + fc[v].s * yc[P][c][2 * v] + fc[v].n * yc[N][c][2 * v];
                    bui -= fc[v].w * uwi + fc[v].e * uei + fc[v].s * yc[P][c][2 * v + 1] +
                           fc[v].n * yc[N][c][2 * v + 1];
                    const R dr = ucr - xc[KC][c][2 * v], di = uci - xc[KC][c][2 * v + 1];
                    const R qr = hc0[c][2 * v] - bur, qi = hc0[c][2 * v + 1] - bui;
                    z[2 * v] = ucr + (ar * dr - ai * di) + (kr * qr - ki * qi);
                    z[2 * v + 1] = uci + (ar * di + ai * dr) + (kr * qi + ki * qr);
                }
                store_row(a.out2, a.soff[s], y, std::integral_constant<int, 2>{}, z);
            }
        }
    };

    auto keep_rhat = [&]() {
#pragma unroll
        for (int v = 0; v < VX; ++v) hr0[v] = hr1[v];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int v = 0; v < 2 * VX; ++v) hc0[c][v] = hc1[c][v];
    };
    auto keep_kappa = [&](auto S_) {
        constexpr int S = decltype(S_)::value;
#pragma unroll
        for (int v = 0; v < VX; ++v) kprev[v] = kw[S][v];
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    // x_k / kappa slot of row r: (r - y0 + 2) mod 3; x_{k+1} slot of row r: (r - y0 + 1) mod 3.
    load_row(I0{}, y0 - 2);
    load_row(I1{}, y0 - 1);
    load_row(I2{}, y0);
    load_centre(y0 - 1);
    step1(I0{}, I1{}, I2{}, I0{}, y0 - 1);
    load_row(I0{}, y0 + 1);
    load_centre(y0);
    step1(I1{}, I2{}, I0{}, I1{}, y0);
    keep_rhat();
    // iteration at row y (i = y - y0): rows y-1, y, y+1 of x_k / kappa sit in slots
    // (i+1, i+2, i) mod 3; row y+2 replaces row y-1.  x_{k+1} rows y-1, y, y+1 sit in
    // slots (i, i+1, i+2) mod 3, row y+1 being computed here.
    int y = y0;
    while (y < y1) {
        keep_kappa(I1{});
        load_row(I1{}, y + 2);
        load_centre(y + 1);
        step1(I2{}, I0{}, I1{}, I2{}, y + 1);
        step2(I0{}, I1{}, I2{}, I2{}, I0{}, y);
        keep_rhat();
        if (++y >= y1) break;
        keep_kappa(I2{});
        load_row(I2{}, y + 2);
        load_centre(y + 1);
        step1(I0{}, I1{}, I2{}, I0{}, y + 1);
        step2(I1{}, I2{}, I0{}, I0{}, I1{}, y);
        keep_rhat();
        if (++y >= y1) break;
        keep_kappa(I0{});
        load_row(I0{}, y + 2);
        load_centre(y + 1);
        step1(I1{}, I2{}, I0{}, I1{}, y + 1);
        step2(I2{}, I0{}, I1{}, I1{}, I2{}, y);
        keep_rhat();
        ++y;
    }
}

template <typename R, typename KS, int VX>
__global__ __launch_bounds__(256) void cheb_pair_kernel(const PairArgs<R> a) {
    cheb_pair_body<R, KS, VX>(a, blockIdx.x, gridDim.x);
}

// Batched: one pair sweep of one shift group for every live problem of a work list
template <typename R, typename KS, int VX>
__global__ __launch_bounds__(256) void cheb_pair_batch_kernel(const BatchList L) {
    const LiveBlocks W = list_live_blocks(L);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const PairArgs<R>& a = list_args<PairArgs<R>>(L.args, q);
        cheb_pair_body<R, KS, VX>(a, local, nb);
    }
}

template <typename R, typename KS>
hipError_t pair_batch_t(int vx, const BatchList& L, hipStream_t s) {
    const dim3 grid(list_grid(L.blocks, L.nprob, L.wpb)), block(L.wpb * kWave);
    if (vx == 2) hipLaunchKernelGGL((cheb_pair_batch_kernel<R, KS, 2>), grid, block, 0, s, L);
    else if (vx == 1) hipLaunchKernelGGL((cheb_pair_batch_kernel<R, KS, 1>), grid, block, 0, s, L);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R, typename KS>
hipError_t pair_launch_t(const void* args, hipStream_t s) {
    const PairArgs<R>& a = *static_cast<const PairArgs<R>*>(args);
    if (a.g.periodic || a.t.blocks <= 0 || a.t.wpb < 1 || a.t.wpb > 4) return hipErrorInvalidValue;
    if (a.t.vx == 2 && a.g.nx % 2 != 0) return hipErrorInvalidValue;
    const dim3 grid(a.t.blocks), block(a.t.wpb * kWave);
    if (a.t.vx == 2) hipLaunchKernelGGL((cheb_pair_kernel<R, KS, 2>), grid, block, 0, s, a);
    else if (a.t.vx == 1) hipLaunchKernelGGL((cheb_pair_kernel<R, KS, 1>), grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cheb_pair(int prec, const void* args, hipStream_t s) {
    switch (prec) {
        case 0: return pair_launch_t<double, double>(args, s);
        case 1: return pair_launch_t<float, uint16_t>(args, s);
        case 2: return pair_launch_t<float, float>(args, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_pair(int prec, int vx, const BatchList& L, hipStream_t s) {
    if (L.nprob < 1 || L.blocks < 1) return hipSuccess;
    if (L.nprob > kListMax || L.wpb < 1 || L.wpb > 4) return hipErrorInvalidValue;
    switch (prec) {
        case 0: return pair_batch_t<double, double>(vx, L, s);
        case 1: return pair_batch_t<float, uint16_t>(vx, L, s);
        case 2: return pair_batch_t<float, float>(vx, L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ac
