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
// windows).  One launch carries every group: a workgroup owns one tile -- a strip of
// 64*VX computed columns and a chunk of h rows -- and holds one wave per group, so the
// waves of a tile march the same rows together and share the tile's kappa rows and
// halos through the caches, and the launch has groups times as many waves as tiles
// (taller chunks for the same occupancy: fewer halo rows per computed row).  Strips
// advance by 64*VX - 4 columns and own the x_{k+2}, x_{k+3} values of their inner
// columns [x0 + 2, x0 + 64*VX - 3] (the first strip from column 0, whose outer
// neighbours are Dirichlet ghosts).  Every point is written by exactly one wave.
// Dirichlet grids only.  Loads are raw buffer loads: lanes past the grid edge, non-halo
// lanes and halo values outside the grid read zeros (the ghosts) without a branch.
//
// The face coefficients of a row are formed once, when its kappa row arrives, and kept
// for the three steps that use the row (a three-row window, like the iterates).  Lanes
// past the grid edge get zero faces, so their iterates stay exactly zero (zero operands,
// zero couplings) without a select; rows outside the grid are skipped by a uniform
// branch.  East / west neighbours cross lanes by DPP wavefront shifts whose vacated lane
// takes the strip-edge halo value (x_k) or zero (the recomputed windows).
//
// Each step evaluates the recurrence with the momentum and the shift folded into one
// complex factor (g u - a x_{k-1} + c (rhat - A' u), below): the same polynomial as the
// single-step sweep, whose iterates it reproduces up to rounding (a few ulps per step).
//
// FIRST: steps 1..3 from a zero initial guess.  x_1 = rhat / theta is never stored: the
// x_k window holds rhat itself (the scale is applied after the linear stencil, as in the
// single first sweep), x_0 = 0, and step 2 takes x_1 = rhat / theta as its x_{k-1}; the
// block reads only rhat and kappa.
#pragma once
#include "stencil_kernels.h"

namespace ac {
namespace {

// XCD-aware tile of a workgroup (block bid of nb; blocks are dealt round-robin to the
// eight XCDs, so XCD x gets a contiguous band of tiles); -1 past the last tile.
__device__ __forceinline__ int tile_of_block(const Tiling& t, int bid, int nb) {
    const int per = nb >> 3;
    const int full = per << 3;
    const int b2 = (bid < full) ? (bid & 7) * per + (bid >> 3) : bid;
    return b2 < t.tiles ? b2 : -1;
}

// Face coefficients of one row for a lane's VX points: the diagonal 1 + w + e + s + n,
// the east face of each point (the west face of point v > 0 is the east face of v - 1),
// the west face of point 0, and the south / north faces.  All zero on lanes past the
// grid edge.
template <typename K, int VX>
struct FaceRow {
    K d[VX], e[VX], s[VX], n[VX];
    K w0;
};

template <typename R, typename KS, int VX, int NS, int NV, bool FIRST>
__device__ __forceinline__ void cheb_triple_body(const TripleArgs<R>& a, const TripleGroup<R>& gp, int tile) {
    using K = R;
    constexpr int W = kWave * VX;  // computed columns per strip
    constexpr int E = NV * VX;     // values per lane and row of one slot

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
    for (int s = 0; s < NS; ++s) comp[s] = gp.comp[s] != 0;

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

    // windows (three rows each, row r in slot (r - y0) mod 3): x_k with its strip-edge
    // halo, x_{k+1}, x_{k+2}, rhat, the faces, kappa in its storage type
    R X[3][NS][E], XH[3][NS][NV];
    R Y[3][NS][E];
    R Z[3][NS][E];
    R H[3][NS][E];
    FaceRow<K, VX> F[3];
    KS KW[3][VX], KH[3];
    R P[NS][E];  // x_{k-1} of the row of step 1

    const unsigned nR = static_cast<unsigned>(sizeof(R));
    const __amdgpu_buffer_rsrc_t rk = buf_rsrc(kap, static_cast<unsigned>(a.g.n) * sizeof(KS));
    const __amdgpu_buffer_rsrc_t rx = buf_rsrc(a.cur, a.bytes);
    const __amdgpu_buffer_rsrc_t rp = buf_rsrc(a.prev, a.bytes);
    const __amdgpu_buffer_rsrc_t rh = buf_rsrc(a.rhat, a.bytes);

    // Row y of x_k (with the strip-edge halo) and kappa into x / xh / kw / kh.  Every load
    // is issued: ghost rows, lanes past the grid, non-halo lanes and slots that do not
    // compute read zeros through an out-of-range offset, so no register needs clearing.
    auto fetch_row = [&](int y, R (&x)[NS][E], R (&xh)[NS][NV], KS (&kw)[VX], KS& kh) {
        const bool row_ok = y >= 0 && y < ny;  // else a Dirichlet ghost row (uniform)
        const unsigned rowp = static_cast<unsigned>(row_ok ? y : 0) * static_cast<unsigned>(nx);
        const unsigned pt = rowp + static_cast<unsigned>(xb);
        const unsigned hp = rowp + static_cast<unsigned>(hx);
        const bool pok = row_ok && lane_ok, qok = row_ok && hok;
        bld<0>(rk, pok ? pt * static_cast<unsigned>(sizeof(KS)) : kOob, kw);
        {
            KS t[1];
            bld<0>(rk, qok ? hp * static_cast<unsigned>(sizeof(KS)) : kOob, t);
            kh = t[0];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const unsigned o = gp.soff[s];
            const __amdgpu_buffer_rsrc_t r = FIRST ? rh : rx;  // FIRST: rhat (x_1 unscaled)
            bld<0>(r, (pok && comp[s]) ? (o + NV * pt) * nR : kOob, x[s]);
            bld<0>(r, (qok && comp[s]) ? (o + NV * hp) * nR : kOob, xh[s]);
        }
    };
    // FIRST blocks read no centre rows, so a row's loads would be waited on at once: they
    // are issued a row ahead into staging registers (rows are requested in order).
    R XS[NS][E], XSH[NS][NV];
    KS KWS[VX], KHS;
    if constexpr (FIRST) fetch_row(y0 - 3, XS, XSH, KWS, KHS);
    auto load_row = [&](auto S_, int y) {
        constexpr int S = decltype(S_)::value;
        if constexpr (FIRST) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
#pragma unroll
                for (int e = 0; e < E; ++e) X[S][s][e] = XS[s][e];
#pragma unroll
                for (int e = 0; e < NV; ++e) XH[S][s][e] = XSH[s][e];
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) KW[S][v] = KWS[v];
            KH[S] = KHS;
            fetch_row(y + 1, XS, XSH, KWS, KHS);
        } else {
            fetch_row(y, X[S], XH[S], KW[S], KH[S]);
        }
    };

    // rhat of row y into h and x_{k-1} into p; non-temporal inside the chunk, plain on its
    // halo rows (also read by the neighbouring chunk).  Not used by FIRST blocks, whose
    // rhat of row y is the x_k window's row y and x_0 = 0.
    auto fetch_centre = [&](int y, R (&h)[NS][E], R (&pv)[NS][E]) {
        const bool row_ok = y >= 0 && y < ny;
        const unsigned pt = static_cast<unsigned>(row_ok ? y : 0) * static_cast<unsigned>(nx) + static_cast<unsigned>(xb);
        const bool inner = (y >= y0 && y < y1);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const unsigned off = (row_ok && lane_ok && comp[s]) ? (gp.soff[s] + NV * pt) * nR : kOob;
            if (inner) {
                bld<2>(rh, off, h[s]);
                bld<2>(rp, off, pv[s]);
            } else {
                bld<0>(rh, off, h[s]);
                bld<0>(rp, off, pv[s]);
            }
        }
    };
    auto load_centre = [&](auto S_, int y) {
        constexpr int S = decltype(S_)::value;
        if constexpr (FIRST) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    H[S][s][e] = X[S][s][e];
                    P[s][e] = R(0);
                }
        } else {
            fetch_centre(y, H[S], P);
        }
    };

    // faces of row y from kappa rows y (kr, halo khr), y-1 (ks), y+1 (kn)
    auto make_faces = [&](FaceRow<K, VX>& f, const KS (&kr)[VX], KS khr, const KS (&ks)[VX], const KS (&kn)[VX],
                          int y) {
        K kc[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) kc[v] = kconv(kr[v]);
        const K khc = kconv(khr);
        const K kwv = from_west(kc[VX - 1], khc);
        const K kev = from_east(kc[0], khc);
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const K kwest = (v > 0) ? kc[v - 1] : kwv;
            const K keast = (v < VX - 1) ? kc[v + 1] : kev;
            const Faces<K> fc = faces<K>(a.g, xb + v, y, kc[v], kwest, keast, kconv(ks[v]), kconv(kn[v]));
            f.d[v] = lane_ok ? fc.diag : K(0);
            f.e[v] = lane_ok ? fc.e : K(0);
            f.s[v] = lane_ok ? fc.s : K(0);
            f.n[v] = lane_ok ? fc.n : K(0);
            if (v == 0) f.w0 = lane_ok ? fc.w : K(0);
        }
    };

    // One Chebyshev step at row y of slot s with the coefficients of step k + T.  The step
    //   x_{k+1} = x_k + a (x_k - x_{k-1}) + c (rhat - (A - lambda) x_k)
    // is evaluated as g u - a xp + c (rh - A' u) with g = 1 + a + c lambda (folded on the
    // host), A' u = d u - sum_f w_f u_nb the real stencil, u the centre window row with
    // south / north rows us / un; the east / west values of the strip-edge lanes are hw /
    // he (the x_k halo, or zero).  FIRST steps 1 and 2 use the same form with the host's
    // scaled coefficients and zero / rhat operands (x_1 = rhat / theta).
    auto update = [&](const FaceRow<K, VX>& f, auto T_, int s, const R (&u)[E], const R (&us)[E], const R (&un)[E],
                      const R* hw, const R* he, const R (&xp)[E], const R (&rhs)[E], R (&out)[E]) {
        constexpr int T = decltype(T_)::value;
        // the strip-edge neighbours: the x_k halo (hw / he), or zero (null)
        auto west = [&](R v, int i) { return hw ? from_west(v, hw[i]) : from_west0(v); };
        auto east = [&](R v, int i) { return he ? from_east(v, he[i]) : from_east0(v); };
        if constexpr (NV == 1) {
            const R wv = west(u[VX - 1], 0);
            const R ev = east(u[0], 0);
            const R gr = gp.g_re[T][s], ar = gp.a_re[T][s], kr = gp.c_re[T][s];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R uw = (v > 0) ? u[v - 1] : wv;
                const R ue = (v < VX - 1) ? u[v + 1] : ev;
                const R fw = (v > 0) ? f.e[v - 1] : f.w0;
                const R uc = u[v];
                const R su = f.d[v] * uc - (fw * uw + f.e[v] * ue + f.s[v] * us[v] + f.n[v] * un[v]);
                out[v] = gr * uc - ar * xp[v] + kr * (rhs[v] - su);
            }
        } else {
            const R wre = west(u[2 * VX - 2], 0);
            const R wim = west(u[2 * VX - 1], 1);
            const R ere = east(u[0], 0);
            const R eim = east(u[1], 1);
            const R gr = gp.g_re[T][s], gi = gp.g_im[T][s];
            const R ar = gp.a_re[T][s], ai = gp.a_im[T][s];
            const R kr = gp.c_re[T][s], ki = gp.c_im[T][s];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const R uwr = (v > 0) ? u[2 * v - 2] : wre;
                const R uwi = (v > 0) ? u[2 * v - 1] : wim;
                const R uer = (v < VX - 1) ? u[2 * v + 2] : ere;
                const R uei = (v < VX - 1) ? u[2 * v + 3] : eim;
                const R fw = (v > 0) ? f.e[v - 1] : f.w0;
                const R ucr = u[2 * v], uci = u[2 * v + 1];
                const R sr = f.d[v] * ucr - (fw * uwr + f.e[v] * uer + f.s[v] * us[2 * v] + f.n[v] * un[2 * v]);
                const R si = f.d[v] * uci - (fw * uwi + f.e[v] * uei + f.s[v] * us[2 * v + 1] + f.n[v] * un[2 * v + 1]);
                const R qr = rhs[2 * v] - sr, qi = rhs[2 * v + 1] - si;
                const R xr = xp[2 * v], xi = xp[2 * v + 1];
                out[2 * v] = (gr * ucr - gi * uci) - (ar * xr - ai * xi) + (kr * qr - ki * qi);
                out[2 * v + 1] = (gr * uci + gi * ucr) - (ar * xi + ai * xr) + (kr * qi + ki * qr);
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

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;

    // step 1 at row y (slots PS, CS, NS_ = rows y-1, y, y+1): the faces of row y into
    // face slot CS, then x_{k+1} of row y from the x_k slots into Y slot CS (rhat H[CS],
    // x_{k-1} P)
    auto step1 = [&](auto PS_, auto CS_, auto NS_, int y) {
        constexpr int PS = decltype(PS_)::value, CS = decltype(CS_)::value, NN = decltype(NS_)::value;
        if (y < 0 || y >= ny) {  // outside the grid (uniform): the ghost row
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < E; ++e) Y[CS][s][e] = R(0);
            return;
        }
        make_faces(F[CS], KW[CS], KH[CS], KW[PS], KW[NN], y);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                if constexpr (FIRST) {  // x_k = rhat / theta, x_{k-1} = 0, the rhat term folded into g
                    const R zr[E] = {};
                    update(F[CS], I0{}, s, X[CS][s], X[PS][s], X[NN][s], XH[CS][s], XH[CS][s], zr, zr, Y[CS][s]);
                } else {
                    update(F[CS], I0{}, s, X[CS][s], X[PS][s], X[NN][s], XH[CS][s], XH[CS][s], P[s], H[CS][s],
                           Y[CS][s]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) Y[CS][s][e] = R(0);
            }
        }
    };

    // step 2 at row y: x_{k+2} from the x_{k+1} slots and x_k of row y (X slot CS), into
    // Z slot CS; stored on the chunk's rows.
    auto step2 = [&](auto PS_, auto CS_, auto NS_, int y) {
        constexpr int PS = decltype(PS_)::value, CS = decltype(CS_)::value, NN = decltype(NS_)::value;
        if (y < 0 || y >= ny) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < E; ++e) Z[CS][s][e] = R(0);
            return;
        }
        const bool st = y >= y0 && y < y1;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                // (FIRST: x_{k-1} = x_1 = rhat / theta, the scale folded into a)
                update(F[CS], I1{}, s, Y[CS][s], Y[PS][s], Y[NN][s], nullptr, nullptr, X[CS][s], H[CS][s], Z[CS][s]);
                if (st) store_row(a.outz, gp.soff[s], y, Z[CS][s]);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) Z[CS][s][e] = R(0);
            }
        }
    };

    // step 3 at row y (a chunk row): x_{k+3} from the x_{k+2} slots and x_{k+1} of row y
    // (Y slot CS); stored.
    auto step3 = [&](auto PS_, auto CS_, auto NS_, int y) {
        constexpr int PS = decltype(PS_)::value, CS = decltype(CS_)::value, NN = decltype(NS_)::value;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (comp[s]) {
                R o[E];
                update(F[CS], I2{}, s, Z[CS][s], Z[PS][s], Z[NN][s], nullptr, nullptr, Y[CS][s], H[CS][s], o);
                store_row(a.outw, gp.soff[s], y, o);
            }
        }
    };

    // Prologue.  Row r lives in slot (r - y0) mod 3 of every window.
    load_row(I0{}, y0 - 3);
    load_row(I1{}, y0 - 2);
    load_row(I2{}, y0 - 1);
    load_centre(I1{}, y0 - 2);
    step1(I0{}, I1{}, I2{}, y0 - 2);  // x_{k+1}(y0-2) -> Y slot 1
    load_row(I0{}, y0);
    load_centre(I2{}, y0 - 1);
    step1(I1{}, I2{}, I0{}, y0 - 1);  // x_{k+1}(y0-1) -> Y slot 2
    load_row(I1{}, y0 + 1);
    load_centre(I0{}, y0);
    step1(I2{}, I0{}, I1{}, y0);      // x_{k+1}(y0) -> Y slot 0
    step2(I1{}, I2{}, I0{}, y0 - 1);  // x_{k+2}(y0-1) -> Z slot 2
    load_row(I2{}, y0 + 2);
    load_centre(I1{}, y0 + 1);
    step1(I0{}, I1{}, I2{}, y0 + 1);  // x_{k+1}(y0+1) -> Y slot 1
    step2(I2{}, I0{}, I1{}, y0);      // x_{k+2}(y0) -> Z slot 0

    // Iteration at row y (i = y - y0): load row y+3 of x_k / kappa and row y+2 of rhat /
    // x_{k-1}, then x_{k+1}(y+2), x_{k+2}(y+1), x_{k+3}(y).  (Loading the steady blocks'
    // rows a row ahead into staging registers was measured slower: with the centre rows
    // 230-270 against 204 us per block at 2048^2, with the x_k / kappa row alone 229
    // against 206 us -- four waves per SIMD instead of five.  FIRST blocks stage their
    // one row: 155 against 170 us.)
    int y = y0;
    while (y < y1) {
        // i = 0 mod 3: rows y-1 .. y+3 in slots 2, 0, 1, 2, 0
        load_row(I0{}, y + 3);
        load_centre(I2{}, y + 2);
        step1(I1{}, I2{}, I0{}, y + 2);
        step2(I0{}, I1{}, I2{}, y + 1);
        step3(I2{}, I0{}, I1{}, y);
        if (++y >= y1) break;
        // i = 1: rows y-1 .. y+3 in slots 0, 1, 2, 0, 1
        load_row(I1{}, y + 3);
        load_centre(I0{}, y + 2);
        step1(I2{}, I0{}, I1{}, y + 2);
        step2(I1{}, I2{}, I0{}, y + 1);
        step3(I0{}, I1{}, I2{}, y);
        if (++y >= y1) break;
        // i = 2: rows y-1 .. y+3 in slots 1, 2, 0, 1, 2
        load_row(I2{}, y + 3);
        load_centre(I1{}, y + 2);
        step1(I0{}, I1{}, I2{}, y + 2);
        step2(I2{}, I0{}, I1{}, y + 1);
        step3(I1{}, I2{}, I0{}, y);
        ++y;
    }
}

// One launch per block of three steps: workgroup = tile, wave = shift group (kind 0: up
// to two real shifts, kind 1: one complex shift; waves past the last group return).
template <typename R, typename KS, int VX, bool FIRST>
__device__ __forceinline__ void cheb_triple_tile(const TripleArgs<R>& a, int tile) {
    const int g = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    if (tile < 0 || g >= a.ngroups) return;
    const TripleGroup<R>& gp = a.grp[g];
    if (gp.kind == 0) cheb_triple_body<R, KS, VX, 2, 1, FIRST>(a, gp, tile);
    else cheb_triple_body<R, KS, VX, 1, 2, FIRST>(a, gp, tile);
}

template <typename R, typename KS, int VX, bool FIRST>
__global__ __launch_bounds__(kWave * kMaxTripleGroups) void cheb_triple_kernel(const TripleArgs<R> a) {
    const int tile = __builtin_amdgcn_readfirstlane(tile_of_block(a.t, blockIdx.x, gridDim.x));
    cheb_triple_tile<R, KS, VX, FIRST>(a, tile);
}

// Batched: problem q owns blocks [first[q], first[q+1]) of the work list (convergence
// mask: a problem whose live flag is zero returns at once).
template <typename R, typename KS, int VX, bool FIRST>
__global__ __launch_bounds__(kWave * kMaxTripleGroups) void cheb_triple_batch_kernel(const BatchList L) {
    const LiveBlocks W = list_live_blocks(L);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const TripleArgs<R>& a = list_args<TripleArgs<R>>(L.args, q);
        cheb_triple_tile<R, KS, VX, FIRST>(a, __builtin_amdgcn_readfirstlane(tile_of_block(a.t, local, nb)));
    }
}

}  // namespace
}  // namespace ac
