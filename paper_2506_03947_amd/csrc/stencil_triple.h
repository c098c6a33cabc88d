// Three steady shifted-Chebyshev steps in one marching sweep (temporal blocking): the
// device body, included by the single-problem and the batched launch files.
//
// Steps k, k+1, k+2 of the three-term recurrence (Section 3) read x_k (stencil), x_{k-1}
// and rhat and write x_{k+2} and x_{k+3}: five vector streams per shift for three steps
// (single steps: twelve; paired steps: 7.5).  x_{k+1} and x_{k+2} are carried in
// three-row register windows; x_{k+1} is recomputed on a two-row / two-column halo of
// the tile and x_{k+2} on a one-row / one-column halo.
//
// A group is one complex shift or up to two real shifts (the register budget of three
// windows).  A wave owns a strip of 64*VX computed columns and a chunk of h rows; strips
// advance by 64*VX - 4 columns and own the x_{k+2}, x_{k+3} values of their inner
// columns [x0 + 2, x0 + 64*VX - 3] (the first strip from column 0, whose outer
// neighbours are Dirichlet ghosts).  Every point is written by exactly one wave.
// Dirichlet grids only.  Loads are raw buffer loads: lanes past the grid edge, non-halo
// lanes and halo values outside the grid read zeros (the ghosts) without a branch.
//
// Arithmetic per point is the single-step sweep's, term for term: the iterates agree with
// three single steps up to rounding (the compiler may contract the same expressions
// differently in another kernel: a few ulps).
//
// FIRST: steps 1..3 from a zero initial guess.  x_1 = rhat / theta is never stored: the
// x_k window holds rhat itself (the scale is applied after the linear stencil, as in the
// single first sweep), x_0 = 0, and step 2 takes x_1 = rhat / theta as its x_{k-1}; the
// block reads only rhat and kappa.
#pragma once
#include "stencil_kernels.h"

namespace ac {
namespace {

template <typename R, typename KS, int VX, int NS, int NV, bool FIRST>
__device__ __forceinline__ void cheb_triple_body(const TripleArgs<R>& a, int bid, int nb) {
    using K = R;
    constexpr int W = kWave * VX;  // computed columns per strip
    constexpr int E = NV * VX;     // values per lane and row of one slot

    const int tile = __builtin_amdgcn_readfirstlane(static_cast<int>(tile_of_wave(a.t, bid, nb)));
    if (tile < 0) return;
    const int nx = a.g.nx, ny = a.g.ny;
    const int lane = threadIdx.x & (kWave - 1);
    const int sx = tile % a.t.nsx;
    const int cy = tile / a.t.nsx;
    const int x0 = sx * (W - 4);
    const int y0 = cy * a.t.h;
    const int y1 = min(y0 + a.t.h, ny);
    const KS* __restrict__ kap = static_cast<const KS*>(a.kappa);

    bool comp[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) comp[s] = a.comp[s] != 0;

    const int xb = x0 + lane * VX;
    const bool lane_ok = xb < nx;  // VX = 2 only on even nx
    const bool hl = (lane == 0 || lane == kWave - 1);
    const int hx = (lane == 0) ? x0 - 1 : x0 + W;
    const bool hok = hl && hx >= 0 && hx < nx;
    bool own[VX];
    bool own_all = true, own_any = false;
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int c = xb + v;
        own[v] = lane_ok && (c >= x0 + 2 || x0 == 0) && c <= x0 + W - 3;
        own_all = own_all && own[v];
        own_any = own_any || own[v];
    }

    // windows (three rows each): x_k with its strip-edge halo, x_{k+1}, x_{k+2}; kappa in
    // its storage type
    R X[3][NS][E], XH[3][NS][NV];
    R Y[3][NS][E];
    R Z[3][NS][E];
    KS KW[3][VX], KH[3];
    KS KF[VX], KFH;  // kappa of row y (with halo), kept for the third step
    KS KB[VX];       // kappa of row y-1
    R H0[NS][E], H1[NS][E], HN[NS][E];  // rhat of rows y, y+1, y+2
    R P[NS][E];                         // x_{k-1} of row y+2

    const unsigned nR = static_cast<unsigned>(sizeof(R));
    const __amdgpu_buffer_rsrc_t rk = buf_rsrc(kap, static_cast<unsigned>(a.g.n) * sizeof(KS));
    const __amdgpu_buffer_rsrc_t rx = buf_rsrc(a.cur, a.bytes);
    const __amdgpu_buffer_rsrc_t rp = buf_rsrc(a.prev, a.bytes);
    const __amdgpu_buffer_rsrc_t rh = buf_rsrc(a.rhat, a.bytes);

    auto load_row = [&](auto S_, int y) {
        constexpr int S = decltype(S_)::value;
#pragma unroll
        for (int v = 0; v < VX; ++v) KW[S][v] = KS(0);
        KH[S] = KS(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int e = 0; e < E; ++e) X[S][s][e] = R(0);
#pragma unroll
            for (int e = 0; e < NV; ++e) XH[S][s][e] = R(0);
        }
        if (y < 0 || y >= ny) return;  // Dirichlet ghost row (uniform)
        const unsigned rowp = static_cast<unsigned>(y) * static_cast<unsigned>(nx);
        const unsigned pt = rowp + static_cast<unsigned>(xb);
        const unsigned hp = rowp + static_cast<unsigned>(hx);
        bld<0>(rk, lane_ok ? pt * static_cast<unsigned>(sizeof(KS)) : kOob, KW[S]);
        {
            KS t[1];
            bld<0>(rk, hok ? hp * static_cast<unsigned>(sizeof(KS)) : kOob, t);
            KH[S] = t[0];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                const unsigned o = a.soff[s];
                const __amdgpu_buffer_rsrc_t r = FIRST ? rh : rx;  // FIRST: rhat (x_1 unscaled)
                bld<0>(r, lane_ok ? (o + NV * pt) * nR : kOob, X[S][s]);
                bld<0>(r, hok ? (o + NV * hp) * nR : kOob, XH[S][s]);
            }
        }
    };

    // rhat into HN and x_{k-1} into P for row y; non-temporal inside the chunk, plain on
    // its halo rows (also read by the neighbouring chunk).  FIRST: rhat of row y is the
    // x_k window's slot XS (already loaded) and x_0 = 0.
    auto load_centre = [&](auto XS_, int y) {
        constexpr int XS = decltype(XS_)::value;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                HN[s][e] = FIRST ? X[XS][s][e] : R(0);
                P[s][e] = R(0);
            }
        if (FIRST || y < 0 || y >= ny) return;
        const unsigned pt = static_cast<unsigned>(y) * static_cast<unsigned>(nx) + static_cast<unsigned>(xb);
        const bool inner = (y >= y0 && y < y1);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                const unsigned off = lane_ok ? (a.soff[s] + NV * pt) * nR : kOob;
                if (inner) {
                    bld<2>(rh, off, HN[s]);
                    bld<2>(rp, off, P[s]);
                } else {
                    bld<0>(rh, off, HN[s]);
                    bld<0>(rp, off, P[s]);
                }
            }
        }
    };

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

    // One Chebyshev step at row y of slot s with coefficients cf:
    //   out = u + a (u - xp) + c (rh - (A - lambda) u),
    // u the centre window row (C) with south / north rows (Sr, Nr); the east / west
    // values of the strip-edge lanes are hw / he (the x_k halo, or zero).
    auto update = [&](const Faces<K> (&fc)[VX], const ShiftCoef<R>& cf, int s, const R (&u)[E], const R (&us)[E],
                      const R (&un)[E], const R (&hw)[NV], const R (&he)[NV], const R (&xp)[E], const R (&rhs)[E],
                      R (&out)[E]) {
        if constexpr (NV == 1) {
            const R wv = shfl_up1(u[VX - 1]);
            const R ev = shfl_dn1(u[0]);
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R uw = (v > 0) ? u[v - 1] : (lane == 0 ? hw[0] : wv);
                const R ue = (v < VX - 1) ? u[v + 1] : (lane == kWave - 1 ? he[0] : ev);
                const R uc = u[v];
                R bu = (fc[v].diag - cf.lam_re[s]) * uc;
                bu -= fc[v].w * uw + fc[v].e * ue + fc[v].s * us[v] + fc[v].n * un[v];
                out[v] = uc + cf.a_re[s] * (uc - xp[v]) + cf.c_re[s] * (rhs[v] - bu);
            }
        } else {
            const R wre = shfl_up1(u[2 * VX - 2]);
            const R wim = shfl_up1(u[2 * VX - 1]);
            const R ere = shfl_dn1(u[0]);
            const R eim = shfl_dn1(u[1]);
            const R lr = cf.lam_re[s], li = cf.lam_im[s];
            const R ar = cf.a_re[s], ai = cf.a_im[s];
            const R kr = cf.c_re[s], ki = cf.c_im[s];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R uwr = (v > 0) ? u[2 * v - 2] : (lane == 0 ? hw[0] : wre);
                const R uwi = (v > 0) ? u[2 * v - 1] : (lane == 0 ? hw[1] : wim);
                const R uer = (v < VX - 1) ? u[2 * v + 2] : (lane == kWave - 1 ? he[0] : ere);
                const R uei = (v < VX - 1) ? u[2 * v + 3] : (lane == kWave - 1 ? he[1] : eim);
                const R ucr = u[2 * v], uci = u[2 * v + 1];
                const R dl = fc[v].diag - lr;
                R bur = dl * ucr + li * uci;
                R bui = dl * uci - li * ucr;
                bur -= fc[v].w * uwr + fc[v].e * uer + fc[v].s * us[2 * v] + fc[v].n * un[2 * v];
                bui -= fc[v].w * uwi + fc[v].e * uei + fc[v].s * us[2 * v + 1] + fc[v].n * un[2 * v + 1];
                const R dr = ucr - xp[2 * v], di = uci - xp[2 * v + 1];
                const R qr = rhs[2 * v] - bur, qi = rhs[2 * v + 1] - bui;
                out[2 * v] = ucr + (ar * dr - ai * di) + (kr * qr - ki * qi);
                out[2 * v + 1] = uci + (ar * di + ai * dr) + (kr * qi + ki * qr);
            }
        }
    };

    // FIRST, step 1: x_2 from x_1 = s rhat (s = 1/theta) and x_0 = 0, the stencil applied
    // to rhat and scaled after (the single first sweep's arithmetic)
    auto update_first = [&](const Faces<K> (&fc)[VX], const ShiftCoef<R>& cf, int s, const R (&u)[E],
                            const R (&us)[E], const R (&un)[E], const R (&hw)[NV], const R (&he)[NV], R (&out)[E]) {
        if constexpr (NV == 1) {
            const R sc = cf.s_re[s];
            const R wv = shfl_up1(u[VX - 1]);
            const R ev = shfl_dn1(u[0]);
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R uw = (v > 0) ? u[v - 1] : (lane == 0 ? hw[0] : wv);
                const R ue = (v < VX - 1) ? u[v + 1] : (lane == kWave - 1 ? he[0] : ev);
                const R uc = u[v];
                R bu = (fc[v].diag - cf.lam_re[s]) * uc;
                bu -= fc[v].w * uw + fc[v].e * ue + fc[v].s * us[v] + fc[v].n * un[v];
                const R xc = sc * uc;
                const R bx = sc * bu;
                const R xp = R(0);
                out[v] = xc + cf.a_re[s] * (xc - xp) + cf.c_re[s] * (uc - bx);
            }
        } else {
            const R sr = cf.s_re[s], si = cf.s_im[s];
            const R wre = shfl_up1(u[2 * VX - 2]);
            const R wim = shfl_up1(u[2 * VX - 1]);
            const R ere = shfl_dn1(u[0]);
            const R eim = shfl_dn1(u[1]);
            const R lr = cf.lam_re[s], li = cf.lam_im[s];
            const R ar = cf.a_re[s], ai = cf.a_im[s];
            const R kr = cf.c_re[s], ki = cf.c_im[s];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R uwr = (v > 0) ? u[2 * v - 2] : (lane == 0 ? hw[0] : wre);
                const R uwi = (v > 0) ? u[2 * v - 1] : (lane == 0 ? hw[1] : wim);
                const R uer = (v < VX - 1) ? u[2 * v + 2] : (lane == kWave - 1 ? he[0] : ere);
                const R uei = (v < VX - 1) ? u[2 * v + 3] : (lane == kWave - 1 ? he[1] : eim);
                const R ucr = u[2 * v], uci = u[2 * v + 1];
                const R dl = fc[v].diag - lr;
                R bur = dl * ucr + li * uci;
                R bui = dl * uci - li * ucr;
                bur -= fc[v].w * uwr + fc[v].e * uer + fc[v].s * us[2 * v] + fc[v].n * un[2 * v];
                bui -= fc[v].w * uwi + fc[v].e * uei + fc[v].s * us[2 * v + 1] + fc[v].n * un[2 * v + 1];
                const R xr = sr * ucr - si * uci, xi = sr * uci + si * ucr;
                const R bxr = sr * bur - si * bui, bxi = sr * bui + si * bur;
                const R xpr = R(0), xpi = R(0);
                const R dr = xr - xpr, di = xi - xpi;
                const R qr = ucr - bxr, qi = uci - bxi;
                out[2 * v] = xr + (ar * dr - ai * di) + (kr * qr - ki * qi);
                out[2 * v + 1] = xi + (ar * di + ai * dr) + (kr * qi + ki * qr);
            }
        }
    };
    // FIRST, step 2: its x_{k-1} is x_1 = s rhat, scaled as the single sweep scales it
    auto scaled_rhat = [&](const ShiftCoef<R>& cf, int s, const R (&u)[E], R (&out)[E]) {
        if constexpr (NV == 1) {
#pragma unroll
            for (int v = 0; v < VX; ++v) out[v] = cf.s_re[s] * u[v];
        } else {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R xpr = u[2 * v], xpi = u[2 * v + 1];
                out[2 * v] = cf.s_re[s] * xpr - cf.s_im[s] * xpi;
                out[2 * v + 1] = cf.s_re[s] * xpi + cf.s_im[s] * xpr;
            }
        }
    };

    auto store_row = [&](R* base, unsigned off, int y, const R (&vals)[E]) {
        if (!own_any) return;
        const unsigned pt = static_cast<unsigned>(y) * static_cast<unsigned>(nx) + static_cast<unsigned>(xb);
        R* d = base + off + static_cast<unsigned>(NV) * pt;
        if (own_all) {
            R t[E];
#pragma unroll
            for (int i = 0; i < E; ++i) t[i] = vals[i];
            stv_nt<R, E>(d, t);
        } else {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                if (own[v]) {
                    R t[NV];
#pragma unroll
                    for (int i = 0; i < NV; ++i) t[i] = vals[NV * v + i];
                    stv<R, NV>(d + NV * v, t);
                }
            }
        }
    };

    const R zh[NV] = {};  // strip-edge neighbour of x_{k+1} / x_{k+2}: not computed (zero)

    // step 1: x_{k+1} of row y from x_k / kappa slots (PS, CS, NS_) = rows (y-1, y, y+1),
    // into x_{k+1} slot YS; rhat HN, x_{k-1} P
    auto step1 = [&](auto PS_, auto CS_, auto NS_, auto YS_, int y) {
        constexpr int PS = decltype(PS_)::value, CS = decltype(CS_)::value, NN = decltype(NS_)::value;
        constexpr int YS = decltype(YS_)::value;
        const bool live = (y >= 0 && y < ny);
        Faces<K> fc[VX];
        row_faces(fc, KW[CS], KH[CS], KW[PS], KW[NN], y);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                R o[E];
                if constexpr (FIRST) update_first(fc, a.cf[0], s, X[CS][s], X[PS][s], X[NN][s], XH[CS][s], XH[CS][s], o);
                else update(fc, a.cf[0], s, X[CS][s], X[PS][s], X[NN][s], XH[CS][s], XH[CS][s], P[s], HN[s], o);
#pragma unroll
                for (int e = 0; e < E; ++e) Y[YS][s][e] = (live && lane_ok) ? o[e] : R(0);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) Y[YS][s][e] = R(0);
            }
        }
    };

    // step 2: x_{k+2} of row y from x_{k+1} slots (PS, CS, NS_) = rows (y-1, y, y+1);
    // x_k of row y is x_k slot XC; faces from kappa row y (kc, with halo), south ks,
    // north kn; rhat rh.  Into x_{k+2} slot ZS; stored on the chunk's rows.
    auto step2 = [&](auto PS_, auto CS_, auto NS_, auto XC_, auto ZS_, const KS (&kc)[VX], KS khc,
                     const KS (&ks)[VX], const KS (&kn)[VX], const R (&rh)[NS][E], int y) {
        constexpr int PS = decltype(PS_)::value, CS = decltype(CS_)::value, NN = decltype(NS_)::value;
        constexpr int XC = decltype(XC_)::value, ZS = decltype(ZS_)::value;
        const bool live = (y >= 0 && y < ny);
        const bool st = live && y >= y0 && y < y1;
        Faces<K> fc[VX];
        row_faces(fc, kc, khc, ks, kn, y);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                R o[E];
                if constexpr (FIRST) {
                    R xp[E];
                    scaled_rhat(a.cf[1], s, X[XC][s], xp);
                    update(fc, a.cf[1], s, Y[CS][s], Y[PS][s], Y[NN][s], zh, zh, xp, rh[s], o);
                } else {
                    update(fc, a.cf[1], s, Y[CS][s], Y[PS][s], Y[NN][s], zh, zh, X[XC][s], rh[s], o);
                }
#pragma unroll
                for (int e = 0; e < E; ++e) Z[ZS][s][e] = (live && lane_ok) ? o[e] : R(0);
                if (st) store_row(a.outz, a.soff[s], y, Z[ZS][s]);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) Z[ZS][s][e] = R(0);
            }
        }
    };

    // step 3: x_{k+3} of row y (a chunk row) from x_{k+2} slots (PS, CS, NS_) = rows
    // (y-1, y, y+1); x_{k+1} of row y is slot YC; kappa row y = KF (with halo), south KB,
    // north slot KN; rhat H0.
    auto step3 = [&](auto PS_, auto CS_, auto NS_, auto YC_, auto KN_, int y) {
        constexpr int PS = decltype(PS_)::value, CS = decltype(CS_)::value, NN = decltype(NS_)::value;
        constexpr int YC = decltype(YC_)::value, KN = decltype(KN_)::value;
        Faces<K> fc[VX];
        row_faces(fc, KF, KFH, KB, KW[KN], y);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                R o[E];
                update(fc, a.cf[2], s, Z[CS][s], Z[PS][s], Z[NN][s], zh, zh, Y[YC][s], H0[s], o);
                store_row(a.outw, a.soff[s], y, o);
            }
        }
    };

    auto copy_rows = [&](R (&dst)[NS][E], const R (&src)[NS][E]) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int e = 0; e < E; ++e) dst[s][e] = src[s][e];
    };
    auto keep_kappa = [&](auto S_) {  // KB <- KF (row y-1), KF <- kappa slot S (row y)
        constexpr int S = decltype(S_)::value;
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            KB[v] = KF[v];
            KF[v] = KW[S][v];
        }
        KFH = KH[S];
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;

    // Prologue.  x_k / kappa slot of row r: (r - y0) mod 3; x_{k+1} slot: (r - y0 + 2)
    // mod 3; x_{k+2} slot: (r - y0 + 1) mod 3.
    R HA[NS][E], HB[NS][E];  // rhat of rows y0-1 and y0
    KS KS2[VX];              // kappa of row y0-2
    load_row(I0{}, y0 - 3);
    load_row(I1{}, y0 - 2);
    load_row(I2{}, y0 - 1);
    load_centre(I1{}, y0 - 2);
    step1(I0{}, I1{}, I2{}, I0{}, y0 - 2);             // x_{k+1}(y0-2) -> Y slot 0
    load_row(I0{}, y0);
    load_centre(I2{}, y0 - 1);
    step1(I1{}, I2{}, I0{}, I1{}, y0 - 1);             // x_{k+1}(y0-1) -> Y slot 1
    copy_rows(HA, HN);
#pragma unroll
    for (int v = 0; v < VX; ++v) KS2[v] = KW[1][v];  // kappa(y0-2) before its slot is reused
    load_row(I1{}, y0 + 1);
    load_centre(I0{}, y0);
    step1(I2{}, I0{}, I1{}, I2{}, y0);                 // x_{k+1}(y0) -> Y slot 2
    copy_rows(HB, HN);
    step2(I0{}, I1{}, I2{}, I2{}, I0{}, KW[2], KH[2], KS2, KW[0], HA, y0 - 1);  // x_{k+2}(y0-1) -> Z slot 0
#pragma unroll
    for (int v = 0; v < VX; ++v) KF[v] = KW[2][v];   // kappa(y0-1) with its halo
    KFH = KH[2];
    load_row(I2{}, y0 + 2);
    load_centre(I1{}, y0 + 1);
    step1(I0{}, I1{}, I2{}, I0{}, y0 + 1);             // x_{k+1}(y0+1) -> Y slot 0
    step2(I1{}, I2{}, I0{}, I0{}, I1{}, KW[0], KH[0], KF, KW[1], HB, y0);  // x_{k+2}(y0) -> Z slot 1
    copy_rows(H0, HB);
    copy_rows(H1, HN);

    // Iteration at row y (i = y - y0): load row y+3 into the slot of row y (after keeping
    // kappa(y)), x_{k+1}(y+2), x_{k+2}(y+1), x_{k+3}(y).
    int y = y0;
    while (y < y1) {
        // i = 0 mod 3: x_k rows y+1, y+2, y+3 in slots 1, 2, 0; x_{k+1} rows y, y+1, y+2
        // in 2, 0, 1; x_{k+2} rows y-1, y, y+1 in 0, 1, 2
        keep_kappa(I0{});
        load_row(I0{}, y + 3);
        load_centre(I2{}, y + 2);
        step1(I1{}, I2{}, I0{}, I1{}, y + 2);
        step2(I2{}, I0{}, I1{}, I1{}, I2{}, KW[1], KH[1], KF, KW[2], H1, y + 1);
        step3(I0{}, I1{}, I2{}, I2{}, I1{}, y);
        copy_rows(H0, H1);
        copy_rows(H1, HN);
        if (++y >= y1) break;
        // i = 1: x_k rows y+1..y+3 in 2, 0, 1; x_{k+1} rows y..y+2 in 0, 1, 2; x_{k+2}
        // rows y-1..y+1 in 1, 2, 0
        keep_kappa(I1{});
        load_row(I1{}, y + 3);
        load_centre(I0{}, y + 2);
        step1(I2{}, I0{}, I1{}, I2{}, y + 2);
        step2(I0{}, I1{}, I2{}, I2{}, I0{}, KW[2], KH[2], KF, KW[0], H1, y + 1);
        step3(I1{}, I2{}, I0{}, I0{}, I2{}, y);
        copy_rows(H0, H1);
        copy_rows(H1, HN);
        if (++y >= y1) break;
        // i = 2: x_k rows y+1..y+3 in 0, 1, 2; x_{k+1} rows y..y+2 in 1, 2, 0; x_{k+2}
        // rows y-1..y+1 in 2, 0, 1
        keep_kappa(I2{});
        load_row(I2{}, y + 3);
        load_centre(I1{}, y + 2);
        step1(I0{}, I1{}, I2{}, I0{}, y + 2);
        step2(I1{}, I2{}, I0{}, I0{}, I1{}, KW[0], KH[0], KF, KW[1], H1, y + 1);
        step3(I2{}, I0{}, I1{}, I1{}, I0{}, y);
        copy_rows(H0, H1);
        copy_rows(H1, HN);
        ++y;
    }
}

template <typename R, typename KS, int VX, int NS, int NV, bool FIRST>
__global__ __launch_bounds__(256) void cheb_triple_kernel(const TripleArgs<R> a) {
    cheb_triple_body<R, KS, VX, NS, NV, FIRST>(a, blockIdx.x, gridDim.x);
}

// Batched: problem q owns blocks [first[q], first[q+1]) of the work list (convergence
// mask: a problem whose live flag is zero returns at once).
template <typename R, typename KS, int VX, int NS, int NV, bool FIRST>
__global__ __launch_bounds__(256) void cheb_triple_batch_kernel(const BatchList L) {
    const int q = batch_problem(L, blockIdx.x);
    if (!L.live[L.pid[q]]) return;
    const TripleArgs<R>& a = static_cast<const TripleArgs<R>*>(L.args)[q];
    cheb_triple_body<R, KS, VX, NS, NV, FIRST>(a, blockIdx.x - L.first[q], L.first[q + 1] - L.first[q]);
}

}  // namespace
}  // namespace ac
