// Marching-stencil kernel templates for gfx950 (included by stencil_ell.hip): the all-at-once operator, the batched
// shifted Chebyshev sweeps, and the scaled time-DFTs.
//
// Every stencil kernel maps one wave (64 lanes) to a strip of 64*VX columns and a
// chunk of H rows.  The wave walks its chunk row by row, holding rows y-1, y, y+1
// of the stencil operand in registers, so each value is read from HBM once per
// sweep (plus the two halo rows of the chunk).  East/west neighbours come from the
// adjacent lane through a cross-lane shuffle; the two strip-edge halo values are
// fetched by lanes 0 and 63 in one extra load per row.  Blocks are remapped so
// that each XCD (blocks are dealt round-robin to the 8 XCDs) owns a contiguous
// band of tiles and the halo rows/columns it shares are hit in its own L2.
//
// Operator (variable-coefficient reading of Section 5, eq. (IminusLap)):
//   (A u)_i = u_i + sum_f kappa_f (u_i - u_nb),  kappa_f = (kappa_i + kappa_nb)/2,
//   Dirichlet boundary face: kappa_f = kappa_i, u_nb = 0;  periodic faces wrap.
#pragma once
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

// ---------------------------------------------------------------------------
// small helpers

template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
    T v[V];
};

template <typename T, int V>
__device__ __forceinline__ void ldv(const T* p, T (&out)[V]) {
    Vec<T, V> t = *reinterpret_cast<const Vec<T, V>*>(p);
#pragma unroll
    for (int i = 0; i < V; ++i) out[i] = t.v[i];
}

template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const T (&in)[V]) {
    Vec<T, V> t;
#pragma unroll
    for (int i = 0; i < V; ++i) t.v[i] = in[i];
    *reinterpret_cast<Vec<T, V>*>(p) = t;
}

// kappa storage -> compute type
__device__ __forceinline__ float kload(const uint16_t* p, long long i) {
    return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
}
__device__ __forceinline__ float kload(const float* p, long long i) { return p[i]; }
__device__ __forceinline__ double kload(const double* p, long long i) { return p[i]; }

template <int V>
__device__ __forceinline__ void kloadv(const uint16_t* p, long long i, float (&o)[V]) {
    uint16_t t[V];
    ldv<uint16_t, V>(p + i, t);
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = __uint_as_float(static_cast<uint32_t>(t[v]) << 16);
}
template <int V>
__device__ __forceinline__ void kloadv(const float* p, long long i, float (&o)[V]) {
    ldv<float, V>(p + i, o);
}
template <int V>
__device__ __forceinline__ void kloadv(const double* p, long long i, double (&o)[V]) {
    ldv<double, V>(p + i, o);
}

__device__ __forceinline__ float shfl_up1(float v) { return __shfl_up(v, 1, kWave); }
__device__ __forceinline__ float shfl_dn1(float v) { return __shfl_down(v, 1, kWave); }
__device__ __forceinline__ double shfl_up1(double v) { return __shfl_up(v, 1, kWave); }
__device__ __forceinline__ double shfl_dn1(double v) { return __shfl_down(v, 1, kWave); }

// XCD-aware tile index of the calling wave; -1 if the wave has no tile.
__device__ __forceinline__ long long tile_of_wave(const Tiling& t) {
    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    const int per = nb >> 3;
    const int full = per << 3;
    const int b2 = (bid < full) ? (bid & 7) * per + (bid >> 3) : bid;
    const long long tile = static_cast<long long>(b2) * t.wpb + (threadIdx.x >> 6);
    return tile < t.tiles ? tile : -1;
}

// Resolves a row index against the grid: returns the row to read, or -1 for a
// Dirichlet ghost row (all zeros).
__device__ __forceinline__ int row_of(const Geom& g, int y) {
    if (y >= 0 && y < g.ny) return y;
    if (!g.periodic) return -1;
    return y < 0 ? y + g.ny : y - g.ny;
}

// Column resolution for periodic / Dirichlet: -1 = zero ghost.
__device__ __forceinline__ int col_of(const Geom& g, int x) {
    if (x >= 0 && x < g.nx) return x;
    if (!g.periodic) return -1;
    int r = x % g.nx;
    return r < 0 ? r + g.nx : r;
}

// One row of a real-valued field: VX points per lane + one halo value
// (lane 0: x0-1, lane 63: x0+64*VX).  Ghost entries are zero.
template <typename T, int VX, typename S>
__device__ __forceinline__ void load_real_row(const S* base, const Geom& g, int y, int x0, int lane, T (&v)[VX],
                                              T& halo) {
    const int yy = row_of(g, y);
    const int xb = x0 + lane * VX;
#pragma unroll
    for (int i = 0; i < VX; ++i) v[i] = T(0);
    halo = T(0);
    if (yy < 0) return;
    const long long rowoff = static_cast<long long>(yy) * g.nx;
    if (xb + VX <= g.nx) {
        T t[VX];
        if constexpr (sizeof(S) == sizeof(T)) {
            ldv<T, VX>(reinterpret_cast<const T*>(base) + rowoff + xb, t);
        } else {
            kloadv<VX>(base, rowoff + xb, t);
        }
#pragma unroll
        for (int i = 0; i < VX; ++i) v[i] = t[i];
    } else if (g.periodic) {
#pragma unroll
        for (int i = 0; i < VX; ++i) v[i] = static_cast<T>(kload(base, rowoff + col_of(g, xb + i)));
    }
    int hx = -1;
    if (lane == 0) hx = col_of(g, x0 - 1);
    if (lane == kWave - 1) hx = col_of(g, x0 + kWave * VX);
    if (hx >= 0) halo = static_cast<T>(kload(base, rowoff + hx));
}

// Complex row (interleaved re, im), scaled by the complex factor (sr, si).
template <typename R, int VX>
__device__ __forceinline__ void load_cplx_row(const R* base, const Geom& g, int y, int x0, int lane, R sr, R si,
                                              R (&re)[VX], R (&im)[VX], R& hre, R& him) {
    const int yy = row_of(g, y);
    const int xb = x0 + lane * VX;
#pragma unroll
    for (int i = 0; i < VX; ++i) re[i] = im[i] = R(0);
    hre = him = R(0);
    if (yy < 0) return;
    const long long rowoff = static_cast<long long>(yy) * g.nx;
    if (xb + VX <= g.nx) {
        R t[2 * VX];
        ldv<R, 2 * VX>(base + 2 * (rowoff + xb), t);
#pragma unroll
        for (int i = 0; i < VX; ++i) {
            re[i] = t[2 * i];
            im[i] = t[2 * i + 1];
        }
    } else if (g.periodic) {
#pragma unroll
        for (int i = 0; i < VX; ++i) {
            const long long o = 2 * (rowoff + col_of(g, xb + i));
            re[i] = base[o];
            im[i] = base[o + 1];
        }
    }
    int hx = -1;
    if (lane == 0) hx = col_of(g, x0 - 1);
    if (lane == kWave - 1) hx = col_of(g, x0 + kWave * VX);
    if (hx >= 0) {
        hre = base[2 * (rowoff + hx)];
        him = base[2 * (rowoff + hx) + 1];
    }
    // apply the scale (identity for buffers)
#pragma unroll
    for (int i = 0; i < VX; ++i) {
        const R a = re[i], b = im[i];
        re[i] = sr * a - si * b;
        im[i] = sr * b + si * a;
    }
    {
        const R a = hre, b = him;
        hre = sr * a - si * b;
        him = sr * b + si * a;
    }
}

// Face coefficients of one point.  kc: own kappa; kw/ke/ks/kn: neighbour kappa
// (ignored where the neighbour is outside a Dirichlet boundary).
template <typename K>
struct Faces {
    K w, e, s, n, diag;
};

template <typename K>
__device__ __forceinline__ Faces<K> faces(const Geom& g, int px, int py, K kc, K kw, K ke, K ks, K kn) {
    Faces<K> f;
    const bool per = g.periodic;
    const K half = K(0.5);
    f.w = (per || px > 0) ? half * (kc + kw) : kc;
    f.e = (per || px < g.nx - 1) ? half * (kc + ke) : kc;
    if (g.dim == 2) {
        f.s = (per || py > 0) ? half * (kc + ks) : kc;
        f.n = (per || py < g.ny - 1) ? half * (kc + kn) : kc;
    } else {
        f.s = K(0);
        f.n = K(0);
    }
    f.diag = K(1) + f.w + f.e + f.s + f.n;
    return f;
}

// ---------------------------------------------------------------------------
// Batched shifted Chebyshev sweep.
//
// For every shift slot with src == SRC_COMPUTE:
//   x_{k+1} = x_k + a (x_k - x_{k-1}) + c (rhat - (A - lambda) x_k)
// The stencil operand x_k is either a buffer (CURK == SRC_BUF) or s * rhat
// (CURK == SRC_RHAT, s = 1/theta: the first iterate from a zero guess).
// x_{k-1} is a buffer (read in place from `out`, or from `prev` in the final
// sweep), s * rhat, or zero.  FINAL fuses the inverse scaled time-DFT: the new
// iterates (and the finished iterates of shifts that stopped earlier) are
// combined in registers into the l float64 blocks of z.

template <typename R, typename KS, int ELL, int VX, int CURK, int PREVK, bool FINAL>
__global__ __launch_bounds__(256) void cheb_sweep_kernel(const SweepArgs<R> a) {
    constexpr int NSR = (ELL % 2 == 0) ? 2 : 1;
    constexpr int NSC = (ELL - NSR) / 2;
    constexpr int NSCA = NSC > 0 ? NSC : 1;  // array extent (l = 2 has no complex shift)
    constexpr int NS = NSR + NSC;
    using K = R;

    const long long tile = tile_of_wave(a.t);
    if (tile < 0) return;
    const Geom& g = a.g;
    const int lane = threadIdx.x & (kWave - 1);
    const int sx = static_cast<int>(tile % a.t.nsx);
    const int cy = static_cast<int>(tile / a.t.nsx);
    const int x0 = sx * kWave * VX;
    const int y0 = cy * a.t.h;
    const int y1 = min(y0 + a.t.h, g.ny);
    const KS* kap = static_cast<const KS*>(a.kappa);

    bool comp[NS];
    bool any = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        comp[s] = (a.src[s] == SRC_COMPUTE);
        any = any || comp[s];
    }

    // three-row windows: p = y-1, c = y, n = y+1
    K kp[VX], kc[VX], kn[VX], khc, khn, kdummy;
    R rp[NSR][VX], rc[NSR][VX], rn[NSR][VX], rhc[NSR], rhn[NSR];
    R cpr[NSCA][VX], cpi[NSCA][VX], ccr[NSCA][VX], cci[NSCA][VX], cnr[NSCA][VX], cni[NSCA][VX];
    R chcr[NSCA], chci[NSCA], chnr[NSCA], chni[NSCA];

    auto load_window_row = [&](int y, K (&kk)[VX], K& kh, R (&rr)[NSR][VX], R (&rh)[NSR], R (&qr)[NSCA][VX],
                               R (&qi)[NSCA][VX], R (&qhr)[NSCA], R (&qhi)[NSCA]) {
        if (any) load_real_row<K, VX, KS>(kap, g, y, x0, lane, kk, kh);
#pragma unroll
        for (int s = 0; s < NSR; ++s) {
            if (comp[s]) {
                const R* src = (CURK == SRC_RHAT) ? a.rhat[s] : a.cur[s];
                load_real_row<R, VX, R>(src, g, y, x0, lane, rr[s], rh[s]);
                if (CURK == SRC_RHAT) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) rr[s][v] *= a.cf.s_re[s];
                    rh[s] *= a.cf.s_re[s];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NSC; ++c) {
            const int s = NSR + c;
            if (comp[s]) {
                const R* src = (CURK == SRC_RHAT) ? a.rhat[s] : a.cur[s];
                const R sr = (CURK == SRC_RHAT) ? a.cf.s_re[s] : R(1);
                const R si = (CURK == SRC_RHAT) ? a.cf.s_im[s] : R(0);
                load_cplx_row<R, VX>(src, g, y, x0, lane, sr, si, qr[c], qi[c], qhr[c], qhi[c]);
            }
        }
    };

    {
        R dr[NSR], dcr[NSCA], dci[NSCA];
        load_window_row(y0 - 1, kp, kdummy, rp, dr, cpr, cpi, dcr, dci);
        load_window_row(y0, kc, khc, rc, rhc, ccr, cci, chcr, chci);
    }

    for (int y = y0; y < y1; ++y) {
        load_window_row(y + 1, kn, khn, rn, rhn, cnr, cni, chnr, chni);

        const long long rowoff = static_cast<long long>(y) * g.nx;
        const int xb = x0 + lane * VX;
        const bool store_ok = (xb < g.nx);

        // kappa neighbours in x
        const K kwv = shfl_up1(kc[VX - 1]);
        const K kev = shfl_dn1(kc[0]);
        Faces<K> fc[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const K kw = (v > 0) ? kc[v - 1] : (lane == 0 ? khc : kwv);
            const K ke = (v < VX - 1) ? kc[v + 1] : (lane == kWave - 1 ? khc : kev);
            fc[v] = faces<K>(g, xb + v, y, kc[v], kw, ke, kp[v], kn[v]);
        }

        // final-sweep accumulators: yhat per slot
        R yr_real[NSR][VX];
        R yc_re[NSCA][VX], yc_im[NSCA][VX];

        // ---- real shifts
#pragma unroll
        for (int s = 0; s < NSR; ++s) {
            if (comp[s]) {
                const R wv = shfl_up1(rc[s][VX - 1]);
                const R ev = shfl_dn1(rc[s][0]);
                R rh[VX], xp[VX];
                if (CURK == SRC_RHAT) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) rh[v] = rc[s][v] / a.cf.s_re[s];
                } else if (store_ok) {
                    ldv<R, VX>(a.rhat[s] + rowoff + xb, rh);
                } else {
#pragma unroll
                    for (int v = 0; v < VX; ++v) rh[v] = R(0);
                }
                if (PREVK == SRC_BUF) {
                    const R* pb = FINAL ? a.prev[s] : a.out[s];
                    if (store_ok) {
                        ldv<R, VX>(pb + rowoff + xb, xp);
                    } else {
#pragma unroll
                        for (int v = 0; v < VX; ++v) xp[v] = R(0);
                    }
                } else if (PREVK == SRC_RHAT) {
                    R t[VX];
                    if (store_ok) {
                        ldv<R, VX>(a.rhat[s] + rowoff + xb, t);
                    } else {
#pragma unroll
                        for (int v = 0; v < VX; ++v) t[v] = R(0);
                    }
#pragma unroll
                    for (int v = 0; v < VX; ++v) xp[v] = a.cf.s_re[s] * t[v];
                } else {
#pragma unroll
                    for (int v = 0; v < VX; ++v) xp[v] = R(0);
                }
                R xo[VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const R xw = (v > 0) ? rc[s][v - 1] : (lane == 0 ? rhc[s] : wv);
                    const R xe = (v < VX - 1) ? rc[s][v + 1] : (lane == kWave - 1 ? rhc[s] : ev);
                    const R xc = rc[s][v];
                    R bx = (fc[v].diag - a.cf.lam_re[s]) * xc;
                    bx -= fc[v].w * xw + fc[v].e * xe + fc[v].s * rp[s][v] + fc[v].n * rn[s][v];
                    xo[v] = xc + a.cf.a_re[s] * (xc - xp[v]) + a.cf.c_re[s] * (rh[v] - bx);
                }
                if (FINAL) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) yr_real[s][v] = xo[v];
                } else if (store_ok) {
                    stv<R, VX>(a.out[s] + rowoff + xb, xo);
                }
            } else if (FINAL) {
                R t[VX];
                if (store_ok) {
                    ldv<R, VX>((a.src[s] == SRC_RHAT ? a.rhat[s] : a.fin[s]) + rowoff + xb, t);
                } else {
#pragma unroll
                    for (int v = 0; v < VX; ++v) t[v] = R(0);
                }
                const R sc = (a.src[s] == SRC_RHAT) ? a.cf.s_re[s] : R(1);
#pragma unroll
                for (int v = 0; v < VX; ++v) yr_real[s][v] = sc * t[v];
            }
        }

        // ---- complex shifts
#pragma unroll
        for (int c = 0; c < NSC; ++c) {
            const int s = NSR + c;
            if (comp[s]) {
                const R wr = shfl_up1(ccr[c][VX - 1]);
                const R wi = shfl_up1(cci[c][VX - 1]);
                const R er = shfl_dn1(ccr[c][0]);
                const R ei = shfl_dn1(cci[c][0]);
                R rhr[VX], rhi[VX], xpr[VX], xpi[VX];
                if (CURK == SRC_RHAT) {
                    // window holds s*rhat; recover rhat = window / s
                    const R sr = a.cf.s_re[s], si = a.cf.s_im[s];
                    const R inv = R(1) / (sr * sr + si * si);
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        rhr[v] = (ccr[c][v] * sr + cci[c][v] * si) * inv;
                        rhi[v] = (cci[c][v] * sr - ccr[c][v] * si) * inv;
                    }
                } else {
                    R t[2 * VX];
                    if (store_ok) {
                        ldv<R, 2 * VX>(a.rhat[s] + 2 * (rowoff + xb), t);
                    } else {
#pragma unroll
                        for (int v = 0; v < 2 * VX; ++v) t[v] = R(0);
                    }
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        rhr[v] = t[2 * v];
                        rhi[v] = t[2 * v + 1];
                    }
                }
                if (PREVK == SRC_BUF) {
                    const R* pb = FINAL ? a.prev[s] : a.out[s];
                    R t[2 * VX];
                    if (store_ok) {
                        ldv<R, 2 * VX>(pb + 2 * (rowoff + xb), t);
                    } else {
#pragma unroll
                        for (int v = 0; v < 2 * VX; ++v) t[v] = R(0);
                    }
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        xpr[v] = t[2 * v];
                        xpi[v] = t[2 * v + 1];
                    }
                } else if (PREVK == SRC_RHAT) {
                    R t[2 * VX];
                    if (store_ok) {
                        ldv<R, 2 * VX>(a.rhat[s] + 2 * (rowoff + xb), t);
                    } else {
#pragma unroll
                        for (int v = 0; v < 2 * VX; ++v) t[v] = R(0);
                    }
                    const R sr = a.cf.s_re[s], si = a.cf.s_im[s];
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        xpr[v] = sr * t[2 * v] - si * t[2 * v + 1];
                        xpi[v] = sr * t[2 * v + 1] + si * t[2 * v];
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < VX; ++v) xpr[v] = xpi[v] = R(0);
                }
                const R lr = a.cf.lam_re[s], li = a.cf.lam_im[s];
                const R ar = a.cf.a_re[s], ai = a.cf.a_im[s];
                const R cr = a.cf.c_re[s], ci = a.cf.c_im[s];
                R xor_[VX], xoi[VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const R xwr = (v > 0) ? ccr[c][v - 1] : (lane == 0 ? chcr[c] : wr);
                    const R xwi = (v > 0) ? cci[c][v - 1] : (lane == 0 ? chci[c] : wi);
                    const R xer = (v < VX - 1) ? ccr[c][v + 1] : (lane == kWave - 1 ? chcr[c] : er);
                    const R xei = (v < VX - 1) ? cci[c][v + 1] : (lane == kWave - 1 ? chci[c] : ei);
                    const R xr = ccr[c][v], xi = cci[c][v];
                    const R dl = fc[v].diag - lr;
                    R bxr = dl * xr + li * xi;
                    R bxi = dl * xi - li * xr;
                    bxr -= fc[v].w * xwr + fc[v].e * xer + fc[v].s * cpr[c][v] + fc[v].n * cnr[c][v];
                    bxi -= fc[v].w * xwi + fc[v].e * xei + fc[v].s * cpi[c][v] + fc[v].n * cni[c][v];
                    const R dr = xr - xpr[v], di = xi - xpi[v];
                    const R qr = rhr[v] - bxr, qi = rhi[v] - bxi;
                    xor_[v] = xr + (ar * dr - ai * di) + (cr * qr - ci * qi);
                    xoi[v] = xi + (ar * di + ai * dr) + (cr * qi + ci * qr);
                }
                if (FINAL) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        yc_re[c][v] = xor_[v];
                        yc_im[c][v] = xoi[v];
                    }
                } else if (store_ok) {
                    R t[2 * VX];
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        t[2 * v] = xor_[v];
                        t[2 * v + 1] = xoi[v];
                    }
                    stv<R, 2 * VX>(a.out[s] + 2 * (rowoff + xb), t);
                }
            } else if (FINAL) {
                R t[2 * VX];
                if (store_ok) {
                    ldv<R, 2 * VX>((a.src[s] == SRC_RHAT ? a.rhat[s] : a.fin[s]) + 2 * (rowoff + xb), t);
                } else {
#pragma unroll
                    for (int v = 0; v < 2 * VX; ++v) t[v] = R(0);
                }
                const bool sc = (a.src[s] == SRC_RHAT);
                const R sr = sc ? a.cf.s_re[s] : R(1), si = sc ? a.cf.s_im[s] : R(0);
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    yc_re[c][v] = sr * t[2 * v] - si * t[2 * v + 1];
                    yc_im[c][v] = sr * t[2 * v + 1] + si * t[2 * v];
                }
            }
        }

        if (FINAL && store_ok) {
            // inverse scaled time-DFT of the l_s unique frequencies (Hermitian
            // symmetry supplies the rest): z_k = ginv_k [y_0 + (-1)^k y_{l/2}
            //   + 2 sum_m (Re y_m cos(2 pi m k/l) - Im y_m sin(2 pi m k/l))]
#pragma unroll
            for (int k = 0; k < ELL; ++k) {
                double zk[VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    double acc = static_cast<double>(yr_real[0][v]);
                    if (NSR == 2) acc += ((k & 1) ? -1.0 : 1.0) * static_cast<double>(yr_real[NSR - 1][v]);
                    double sum = 0.0;
#pragma unroll
                    for (int c = 0; c < NSC; ++c) {
                        const int j = ((c + 1) * k) % ELL;
                        sum += static_cast<double>(yc_re[c][v]) * a.cw[j] - static_cast<double>(yc_im[c][v]) * a.sw[j];
                    }
                    zk[v] = a.ginv[k] * (acc + 2.0 * sum);
                }
                stv<double, VX>(a.z + static_cast<long long>(k) * g.n + rowoff + xb, zk);
            }
        }

        // rotate windows
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            kp[v] = kc[v];
            kc[v] = kn[v];
        }
        khc = khn;
#pragma unroll
        for (int s = 0; s < NSR; ++s) {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                rp[s][v] = rc[s][v];
                rc[s][v] = rn[s][v];
            }
            rhc[s] = rhn[s];
        }
#pragma unroll
        for (int c = 0; c < NSC; ++c) {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                cpr[c][v] = ccr[c][v];
                cpi[c][v] = cci[c][v];
                ccr[c][v] = cnr[c][v];
                cci[c][v] = cni[c][v];
            }
            chcr[c] = chnr[c];
            chci[c] = chni[c];
        }
    }
}

// ---------------------------------------------------------------------------
// Forward scaled time-DFT: per grid point, t_k = gam_k r_k and
// rhat_m = sum_k t_k exp(-2 pi i m k / l) for the l_s unique m, in float64,
// stored in the inner real type.

template <typename R, int ELL, int VX>
__global__ __launch_bounds__(256) void tdft_fwd_kernel(const FwdArgs a) {
    constexpr int NSR = (ELL % 2 == 0) ? 2 : 1;
    constexpr int NSC = (ELL - NSR) / 2;
    constexpr int NSCA = NSC > 0 ? NSC : 1;  // array extent (l = 2 has no complex shift)
    const long long i0 = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) * VX;
    if (i0 >= a.n) return;
    double t[ELL][VX];
#pragma unroll
    for (int k = 0; k < ELL; ++k) {
        double v[VX];
        ldv<double, VX>(a.r + static_cast<long long>(k) * a.n + i0, v);
#pragma unroll
        for (int x = 0; x < VX; ++x) t[k][x] = a.gam[k] * v[x];
    }
    // real slots
    {
        R o0[VX], o1[VX];
#pragma unroll
        for (int x = 0; x < VX; ++x) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < ELL; ++k) {
                s0 += t[k][x];
                s1 += (k & 1) ? -t[k][x] : t[k][x];
            }
            o0[x] = static_cast<R>(s0);
            o1[x] = static_cast<R>(s1);
        }
        stv<R, VX>(static_cast<R*>(a.rhat[0]) + i0, o0);
        if (NSR == 2) stv<R, VX>(static_cast<R*>(a.rhat[1]) + i0, o1);
    }
#pragma unroll
    for (int c = 0; c < NSC; ++c) {
        const int m = c + 1;
        R o[2 * VX];
#pragma unroll
        for (int x = 0; x < VX; ++x) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < ELL; ++k) {
                const int j = (m * k) % ELL;
                re += t[k][x] * a.cw[j];
                im -= t[k][x] * a.sw[j];
            }
            o[2 * x] = static_cast<R>(re);
            o[2 * x + 1] = static_cast<R>(im);
        }
        stv<R, 2 * VX>(static_cast<R*>(a.rhat[NSR + c]) + 2 * i0, o);
    }
}

// Inverse scaled time-DFT (standalone stage).
template <typename R, int ELL, int VX>
__global__ __launch_bounds__(256) void tdft_inv_kernel(const InvArgs a) {
    constexpr int NSR = (ELL % 2 == 0) ? 2 : 1;
    constexpr int NSC = (ELL - NSR) / 2;
    constexpr int NSCA = NSC > 0 ? NSC : 1;  // array extent (l = 2 has no complex shift)
    const long long i0 = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) * VX;
    if (i0 >= a.n) return;
    double yr[NSR][VX], ycr[NSCA][VX], yci[NSCA][VX];
#pragma unroll
    for (int s = 0; s < NSR; ++s) {
        R t[VX];
        ldv<R, VX>(static_cast<const R*>(a.yhat[s]) + i0, t);
#pragma unroll
        for (int x = 0; x < VX; ++x) yr[s][x] = static_cast<double>(t[x]);
    }
#pragma unroll
    for (int c = 0; c < NSC; ++c) {
        R t[2 * VX];
        ldv<R, 2 * VX>(static_cast<const R*>(a.yhat[NSR + c]) + 2 * i0, t);
#pragma unroll
        for (int x = 0; x < VX; ++x) {
            ycr[c][x] = static_cast<double>(t[2 * x]);
            yci[c][x] = static_cast<double>(t[2 * x + 1]);
        }
    }
#pragma unroll
    for (int k = 0; k < ELL; ++k) {
        double zk[VX];
#pragma unroll
        for (int x = 0; x < VX; ++x) {
            double acc = yr[0][x];
            if (NSR == 2) acc += ((k & 1) ? -1.0 : 1.0) * yr[NSR - 1][x];
            double sum = 0.0;
#pragma unroll
            for (int c = 0; c < NSC; ++c) {
                const int j = ((c + 1) * k) % ELL;
                sum += ycr[c][x] * a.cw[j] - yci[c][x] * a.sw[j];
            }
            zk[x] = a.ginv[k] * (acc + 2.0 * sum);
        }
        stv<double, VX>(a.z + static_cast<long long>(k) * a.n + i0, zk);
    }
}

// ---------------------------------------------------------------------------
// All-at-once operator, float64:  y_k = A x_k - x_{k-1} (x_0 := 0), or in
// residual mode y = b - calA x together with per-tile sums of y^2.

template <int ELL, int VX, bool RESID>
__global__ __launch_bounds__(256) void apply_calA_kernel(const CalAArgs a) {
    const long long tile = tile_of_wave(a.t);
    const int lane = threadIdx.x & (kWave - 1);
    double ssq = 0.0;
    if (tile >= 0) {
        const Geom& g = a.g;
        const int sx = static_cast<int>(tile % a.t.nsx);
        const int cy = static_cast<int>(tile / a.t.nsx);
        const int x0 = sx * kWave * VX;
        const int y0 = cy * a.t.h;
        const int y1 = min(y0 + a.t.h, g.ny);

        double kp[VX], kc[VX], kn[VX], khc, khn, kd;
        double xp[ELL][VX], xc[ELL][VX], xn[ELL][VX], hc[ELL], hn[ELL], hd;
        load_real_row<double, VX, double>(a.kappa, g, y0 - 1, x0, lane, kp, kd);
        load_real_row<double, VX, double>(a.kappa, g, y0, x0, lane, kc, khc);
#pragma unroll
        for (int k = 0; k < ELL; ++k) {
            load_real_row<double, VX, double>(a.x + k * g.n, g, y0 - 1, x0, lane, xp[k], hd);
            load_real_row<double, VX, double>(a.x + k * g.n, g, y0, x0, lane, xc[k], hc[k]);
        }
        for (int y = y0; y < y1; ++y) {
            load_real_row<double, VX, double>(a.kappa, g, y + 1, x0, lane, kn, khn);
#pragma unroll
            for (int k = 0; k < ELL; ++k)
                load_real_row<double, VX, double>(a.x + k * g.n, g, y + 1, x0, lane, xn[k], hn[k]);

            const long long rowoff = static_cast<long long>(y) * g.nx;
            const int xb = x0 + lane * VX;
            const bool store_ok = xb < g.nx;
            const double kwv = shfl_up1(kc[VX - 1]);
            const double kev = shfl_dn1(kc[0]);
            Faces<double> fc[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const double kw = (v > 0) ? kc[v - 1] : (lane == 0 ? khc : kwv);
                const double ke = (v < VX - 1) ? kc[v + 1] : (lane == kWave - 1 ? khc : kev);
                fc[v] = faces<double>(g, xb + v, y, kc[v], kw, ke, kp[v], kn[v]);
            }
#pragma unroll
            for (int k = 0; k < ELL; ++k) {
                const double wv = shfl_up1(xc[k][VX - 1]);
                const double ev = shfl_dn1(xc[k][0]);
                double yo[VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const double xw = (v > 0) ? xc[k][v - 1] : (lane == 0 ? hc[k] : wv);
                    const double xe = (v < VX - 1) ? xc[k][v + 1] : (lane == kWave - 1 ? hc[k] : ev);
                    double ax = fc[v].diag * xc[k][v];
                    ax -= fc[v].w * xw + fc[v].e * xe + fc[v].s * xp[k][v] + fc[v].n * xn[k][v];
                    if (k > 0) ax -= xc[k - 1][v];
                    yo[v] = ax;
                }
                if (store_ok) {
                    if (RESID) {
                        double bb[VX];
                        ldv<double, VX>(a.b + k * g.n + rowoff + xb, bb);
#pragma unroll
                        for (int v = 0; v < VX; ++v) {
                            yo[v] = bb[v] - yo[v];
                            ssq += yo[v] * yo[v];
                        }
                    }
                    stv<double, VX>(a.y + k * g.n + rowoff + xb, yo);
                }
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                kp[v] = kc[v];
                kc[v] = kn[v];
            }
            khc = khn;
#pragma unroll
            for (int k = 0; k < ELL; ++k) {
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    xp[k][v] = xc[k][v];
                    xc[k][v] = xn[k][v];
                }
                hc[k] = hn[k];
            }
        }
    }
    if (RESID) {
        // wave sum, lane 0 writes the tile partial
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) ssq += __shfl_down(ssq, off, kWave);
        if (lane == 0 && tile >= 0) a.partial[tile] = ssq;
    }
}

}  // namespace
}  // namespace ac
