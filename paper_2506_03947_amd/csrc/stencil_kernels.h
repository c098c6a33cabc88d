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

#include <type_traits>

#include "ac_internal.h"
#include "worklist.h"

namespace ac {
// Every operand pointer of these kernels addresses global memory.  Saying so lets the
// compiler use global rather than flat memory instructions also when the pointer
// comes from an argument record in memory (batched launches), not from the kernel
// arguments.
template <typename T>
__device__ __forceinline__ T* gptr(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)p;
}
}  // namespace ac

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

// Non-temporal variants for operands touched once per sweep (clang ext vectors).
template <typename T, int V>
using ExtVec = T __attribute__((ext_vector_type(V)));

template <typename T, int V>
__device__ __forceinline__ void ldv_nt(const T* p, T (&out)[V]) {
    if constexpr (V == 1) {
        out[0] = __builtin_nontemporal_load(p);
    } else {
        const ExtVec<T, V> t = __builtin_nontemporal_load(reinterpret_cast<const ExtVec<T, V>*>(p));
#pragma unroll
        for (int i = 0; i < V; ++i) out[i] = t[i];
    }
}

template <typename T, int V>
__device__ __forceinline__ void stv_nt(T* p, const T (&in)[V]) {
    if constexpr (V == 1) {
        __builtin_nontemporal_store(in[0], p);
    } else {
        ExtVec<T, V> t;
#pragma unroll
        for (int i = 0; i < V; ++i) t[i] = in[i];
        __builtin_nontemporal_store(t, reinterpret_cast<ExtVec<T, V>*>(p));
    }
}

// 1: the centre operands (rhat, x_{k-1}) and the new iterate, each touched once per
// sweep, use non-temporal loads/stores (measured +20 % on 2048^2, l = 10, complex64);
// 2: the stencil window as well (slower: the chunk halo rows are then refetched).
#ifndef AC_SWEEP_NT
#define AC_SWEEP_NT 1
#endif
template <typename T, int V>
__device__ __forceinline__ void ldc(const T* p, T (&out)[V]) {
    if constexpr (AC_SWEEP_NT != 0) ldv_nt<T, V>(p, out);
    else ldv<T, V>(p, out);
}
// stencil-window operand (read once per sweep apart from the chunk halo rows)
template <typename T, int V>
__device__ __forceinline__ void ldw(const T* p, T (&out)[V]) {
    if constexpr (AC_SWEEP_NT >= 2) ldv_nt<T, V>(p, out);
    else ldv<T, V>(p, out);
}
template <typename T, int V>
__device__ __forceinline__ void stc(T* p, const T (&in)[V]) {
    if constexpr (AC_SWEEP_NT != 0) stv_nt<T, V>(p, in);
    else stv<T, V>(p, in);
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

// kappa storage value -> compute type (bf16: the high half of a float32)
__device__ __forceinline__ float kconv(uint16_t v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
__device__ __forceinline__ float kconv(float v) { return v; }
__device__ __forceinline__ double kconv(double v) { return v; }

// Raw buffer loads (buffer resource with a byte range): a lane whose byte offset lies
// past the range reads zeros and touches no memory, which gives ghost values without a
// lane-divergent branch.  kOob is such an offset for every range below 2^31 bytes.
constexpr unsigned kOob = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), 0x00020000);
}

// V values of type T at byte offset off; AUX 2 = non-temporal
template <int AUX, typename T, int V>
__device__ __forceinline__ void bld(__amdgpu_buffer_rsrc_t r, unsigned off, T (&out)[V]) {
    constexpr int B = static_cast<int>(sizeof(T)) * V;
    if constexpr (B == 2) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, AUX);
        __builtin_memcpy(out, &u, 2);
    } else if constexpr (B == 4) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX);
        __builtin_memcpy(out, &u, 4);
    } else if constexpr (B == 8) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
        __builtin_memcpy(out, &u, 8);
    } else if constexpr (B == 16) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
        __builtin_memcpy(out, &u, 16);
    } else {
        static_assert(B == 32, "buffer load of 2, 4, 8, 16 or 32 bytes");
        const auto u0 = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
        const auto u1 = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, AUX);
        __builtin_memcpy(out, &u0, 16);
        __builtin_memcpy(reinterpret_cast<char*>(out) + 16, &u1, 16);
    }
}

__device__ __forceinline__ float shfl_up1(float v) { return __shfl_up(v, 1, kWave); }
__device__ __forceinline__ float shfl_dn1(float v) { return __shfl_down(v, 1, kWave); }
__device__ __forceinline__ double shfl_up1(double v) { return __shfl_up(v, 1, kWave); }
__device__ __forceinline__ double shfl_dn1(double v) { return __shfl_down(v, 1, kWave); }

// Wavefront shifts by one lane (DPP): from_west(v, edge) gives lane i the value of lane
// i-1 and lane 0 `edge`; from_east(v, edge) gives lane i the value of lane i+1 and lane
// 63 `edge`.
__device__ __forceinline__ float from_west(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_east(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
// The same with a zero edge value (bound_ctrl: the vacated lane reads zero)
__device__ __forceinline__ float from_west0(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_east0(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_west0(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x138, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ double from_east0(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ double from_west(double v, double edge) {
    const long long b = __builtin_bit_cast(long long, v), e = __builtin_bit_cast(long long, edge);
    const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(e), static_cast<int>(b), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(e >> 32), static_cast<int>(b >> 32), 0x138, 0xf, 0xf,
                                               false);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ double from_east(double v, double edge) {
    const long long b = __builtin_bit_cast(long long, v), e = __builtin_bit_cast(long long, edge);
    const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(e), static_cast<int>(b), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(e >> 32), static_cast<int>(b >> 32), 0x130, 0xf, 0xf,
                                               false);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// XCD-aware tile index of the calling wave (block bid of nb); -1 if the wave has no tile.
__device__ __forceinline__ long long tile_of_wave(const Tiling& t, int bid, int nb) {
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
//   x_{k+1} = x_k + a (x_k - x_{k-1}) + c (rhat - (A - lambda) x_k).
// CUR_RHAT: the stencil operand is x_1 = s * rhat (s = 1/theta, zero initial
// guess, never stored); the window then holds rhat itself and the scale is
// applied after the (linear) stencil.  x_{k-1} is a buffer, s * rhat or zero
// (runtime kind, uniform).  FINAL fuses the inverse scaled time-DFT: the new
// iterates and the finished iterates of shifts that stopped earlier are combined
// in registers into the l float64 blocks of z.
//
// Per row, every load of every shift is issued before the first arithmetic
// instruction that needs one of them (loads complete in order, so each shift
// only waits for its own operands), and all addresses are 32-bit offsets from a
// few uniform base pointers.

template <typename R, typename KS, int ELL, int VX, bool CUR_RHAT, bool FINAL, bool PER>
__device__ __forceinline__ void cheb_sweep_body(const SweepArgs<R>& a, int bid, int nb) {
    constexpr int NSR = (ELL % 2 == 0) ? 2 : 1;
    constexpr int NSC = (ELL - NSR) / 2;
    constexpr int NSCA = NSC > 0 ? NSC : 1;  // array extent (l = 2 has no complex shift)
    constexpr int NS = NSR + NSC;
    using K = R;

    const long long tile = tile_of_wave(a.t, bid, nb);
    if (tile < 0) return;
    const int nx = a.g.nx, ny = a.g.ny;
    const int lane = threadIdx.x & (kWave - 1);
    const int sx = static_cast<int>(tile % a.t.nsx);
    const int cy = static_cast<int>(tile / a.t.nsx);
    const int x0 = sx * kWave * VX;
    const int y0 = cy * a.t.h;
    const int y1 = min(y0 + a.t.h, ny);
    const KS* __restrict__ kap = gptr(static_cast<const KS*>(a.kappa));
    const R* __restrict__ rhat = gptr(a.rhat);

    bool comp[NS];
    bool any = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        comp[s] = (a.src[s] == SRC_COMPUTE);
        any = any || comp[s];
    }
    const R* __restrict__ wbase = gptr(CUR_RHAT ? a.rhat : a.cur);  // stencil operand buffer

    // per-lane columns
    const int xb = x0 + lane * VX;
    const bool lane_ok = PER || (xb < nx);
    const int xl = PER ? (xb % nx) : xb;
    const bool hl = (lane == 0 || lane == kWave - 1);  // lanes that fetch the strip halo
    int hx = -1;
    if (hl) {
        hx = (lane == 0) ? x0 - 1 : x0 + kWave * VX;
        if (PER) hx = ((hx % nx) + nx) % nx;
    }
    const bool hok = hl && hx >= 0 && hx < nx;

    // three-row windows of the stencil operand (raw rhat when CUR_RHAT)
    K kw[3][VX], kh[3];
    R wr[3][NSR][VX], wrh[3][NSR];
    R wc[3][NSCA][2 * VX], wch[3][NSCA][2];

    auto load_row = [&](auto W_, int y) {
        constexpr int W = decltype(W_)::value;
#pragma unroll
        for (int v = 0; v < VX; ++v) kw[W][v] = K(0);
        kh[W] = K(0);
#pragma unroll
        for (int s = 0; s < NSR; ++s) {
#pragma unroll
            for (int v = 0; v < VX; ++v) wr[W][s][v] = R(0);
            wrh[W][s] = R(0);
        }
#pragma unroll
        for (int c = 0; c < NSCA; ++c) {
#pragma unroll
            for (int v = 0; v < 2 * VX; ++v) wc[W][c][v] = R(0);
            wch[W][c][0] = wch[W][c][1] = R(0);
        }
        int yy = y;
        if (PER) yy = (y < 0) ? y + ny : (y >= ny ? y - ny : y);
        if (!PER && (y < 0 || y >= ny)) return;  // Dirichlet ghost row: zeros
        const unsigned rowp = static_cast<unsigned>(yy) * static_cast<unsigned>(nx);
        const unsigned pt = rowp + static_cast<unsigned>(xl);
        const unsigned hp = rowp + static_cast<unsigned>(hx);
        if (any) {
            if (lane_ok) {
                if constexpr (sizeof(KS) == sizeof(K)) {
                    ldv<K, VX>(reinterpret_cast<const K*>(kap) + pt, kw[W]);
                } else {
                    kloadv<VX>(kap, pt, kw[W]);
                }
            }
            if (hok) kh[W] = static_cast<K>(kload(kap, hp));
        }
#pragma unroll
        for (int s = 0; s < NSR; ++s) {
            if (comp[s]) {
                const R* b = wbase + a.soff[s];
                if (lane_ok) ldw<R, VX>(b + pt, wr[W][s]);
                if (hok) wrh[W][s] = b[hp];
            }
        }
#pragma unroll
        for (int c = 0; c < NSC; ++c) {
            if (comp[NSR + c]) {
                const R* b = wbase + a.soff[NSR + c];
                if (lane_ok) ldw<R, 2 * VX>(b + 2u * pt, wc[W][c]);
                if (hok) {
                    wch[W][c][0] = b[2u * hp];
                    wch[W][c][1] = b[2u * hp + 1u];
                }
            }
        }
    };

    // centre-row operands: rhat (unless CUR_RHAT), x_{k-1}, or (FINAL) finished iterates
    R hr[NSR][VX], hc[NSCA][2 * VX];  // rhat centre
    R pr[NSR][VX], pc[NSCA][2 * VX];  // x_{k-1} centre, or finished iterate
    const int prevk = a.prevk;
    const R* __restrict__ pbase = gptr(a.prev);

    auto load_centre = [&](int y) {
        const unsigned pt = static_cast<unsigned>(y) * static_cast<unsigned>(nx) + static_cast<unsigned>(xb);
        const bool ok = (xb < nx);
#pragma unroll
        for (int s = 0; s < NSR; ++s) {
#pragma unroll
            for (int v = 0; v < VX; ++v) hr[s][v] = pr[s][v] = R(0);
            const unsigned o = a.soff[s] + pt;
            if (comp[s]) {
                if (!CUR_RHAT && ok) ldc<R, VX>(rhat + o, hr[s]);
                if (prevk == SRC_BUF && ok) ldc<R, VX>(pbase + o, pr[s]);
                if (prevk == SRC_RHAT && ok) ldc<R, VX>(rhat + o, pr[s]);
            } else if (FINAL && ok) {
                const R* f = gptr((a.src[s] == SRC_RHAT) ? a.rhat : a.bufs[a.fbuf[s]]);
                ldc<R, VX>(f + o, pr[s]);
            }
        }
#pragma unroll
        for (int c = 0; c < NSC; ++c) {
            const int s = NSR + c;
#pragma unroll
            for (int v = 0; v < 2 * VX; ++v) hc[c][v] = pc[c][v] = R(0);
            const unsigned o = a.soff[s] + 2u * pt;
            if (comp[s]) {
                if (!CUR_RHAT && ok) ldc<R, 2 * VX>(rhat + o, hc[c]);
                if (prevk == SRC_BUF && ok) ldc<R, 2 * VX>(pbase + o, pc[c]);
                if (prevk == SRC_RHAT && ok) ldc<R, 2 * VX>(rhat + o, pc[c]);
            } else if (FINAL && ok) {
                const R* f = gptr((a.src[s] == SRC_RHAT) ? a.rhat : a.bufs[a.fbuf[s]]);
                ldc<R, 2 * VX>(f + o, pc[c]);
            }
        }
    };

    auto compute_row = [&](auto P_, auto C_, auto N_, int y) {
        constexpr int P = decltype(P_)::value, C = decltype(C_)::value, N = decltype(N_)::value;
        const unsigned pt = static_cast<unsigned>(y) * static_cast<unsigned>(nx) + static_cast<unsigned>(xb);
        const bool store_ok = (xb < nx);

        // face coefficients, shared by all shifts
        const K kwv = shfl_up1(kw[C][VX - 1]);
        const K kev = shfl_dn1(kw[C][0]);
        Faces<K> fc[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const K kwest = (v > 0) ? kw[C][v - 1] : (lane == 0 ? kh[C] : kwv);
            const K keast = (v < VX - 1) ? kw[C][v + 1] : (lane == kWave - 1 ? kh[C] : kev);
            fc[v] = faces<K>(a.g, xb + v, y, kw[C][v], kwest, keast, kw[P][v], kw[N][v]);
        }

        R yr[NSR][VX];
        R yc[NSCA][2 * VX];

        // ---- real shifts
#pragma unroll
        for (int s = 0; s < NSR; ++s) {
            if (comp[s]) {
                const R sc = CUR_RHAT ? a.cf.s_re[s] : R(1);
                const R wv = shfl_up1(wr[C][s][VX - 1]);
                const R ev = shfl_dn1(wr[C][s][0]);
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const R uw = (v > 0) ? wr[C][s][v - 1] : (lane == 0 ? wrh[C][s] : wv);
                    const R ue = (v < VX - 1) ? wr[C][s][v + 1] : (lane == kWave - 1 ? wrh[C][s] : ev);
                    const R uc = wr[C][s][v];
                    R bu = (fc[v].diag - a.cf.lam_re[s]) * uc;
                    bu -= fc[v].w * uw + fc[v].e * ue + fc[v].s * wr[P][s][v] + fc[v].n * wr[N][s][v];
                    const R xc = sc * uc;
                    const R bx = sc * bu;
                    const R rh = CUR_RHAT ? uc : hr[s][v];
                    const R xp = (prevk == SRC_RHAT) ? a.cf.s_re[s] * pr[s][v] : pr[s][v];
                    yr[s][v] = xc + a.cf.a_re[s] * (xc - xp) + a.cf.c_re[s] * (rh - bx);
                }
                if (!FINAL && store_ok) stc<R, VX>(gptr(a.out) + a.soff[s] + pt, yr[s]);
            } else if (FINAL) {
                const R sc = (a.src[s] == SRC_RHAT) ? a.cf.s_re[s] : R(1);
#pragma unroll
                for (int v = 0; v < VX; ++v) yr[s][v] = sc * pr[s][v];
            }
        }

        // ---- complex shifts
#pragma unroll
        for (int c = 0; c < NSC; ++c) {
            const int s = NSR + c;
            if (comp[s]) {
                const R sr = CUR_RHAT ? a.cf.s_re[s] : R(1);
                const R si = CUR_RHAT ? a.cf.s_im[s] : R(0);
                const R wre = shfl_up1(wc[C][c][2 * VX - 2]);
                const R wim = shfl_up1(wc[C][c][2 * VX - 1]);
                const R ere = shfl_dn1(wc[C][c][0]);
                const R eim = shfl_dn1(wc[C][c][1]);
                const R lr = a.cf.lam_re[s], li = a.cf.lam_im[s];
                const R ar = a.cf.a_re[s], ai = a.cf.a_im[s];
                const R cr = a.cf.c_re[s], ci = a.cf.c_im[s];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const R uwr = (v > 0) ? wc[C][c][2 * v - 2] : (lane == 0 ? wch[C][c][0] : wre);
                    const R uwi = (v > 0) ? wc[C][c][2 * v - 1] : (lane == 0 ? wch[C][c][1] : wim);
                    const R uer = (v < VX - 1) ? wc[C][c][2 * v + 2] : (lane == kWave - 1 ? wch[C][c][0] : ere);
                    const R uei = (v < VX - 1) ? wc[C][c][2 * v + 3] : (lane == kWave - 1 ? wch[C][c][1] : eim);
                    const R ucr = wc[C][c][2 * v], uci = wc[C][c][2 * v + 1];
                    const R dl = fc[v].diag - lr;
                    R bur = dl * ucr + li * uci;
                    R bui = dl * uci - li * ucr;
                    bur -= fc[v].w * uwr + fc[v].e * uer + fc[v].s * wc[P][c][2 * v] + fc[v].n * wc[N][c][2 * v];
                    bui -= fc[v].w * uwi + fc[v].e * uei + fc[v].s * wc[P][c][2 * v + 1] +
                           fc[v].n * wc[N][c][2 * v + 1];
                    // x = s u, B x = s (B u)
                    const R xr = sr * ucr - si * uci, xi = sr * uci + si * ucr;
                    const R bxr = sr * bur - si * bui, bxi = sr * bui + si * bur;
                    const R rhr = CUR_RHAT ? ucr : hc[c][2 * v];
                    const R rhi = CUR_RHAT ? uci : hc[c][2 * v + 1];
                    R xpr = pc[c][2 * v], xpi = pc[c][2 * v + 1];
                    if (prevk == SRC_RHAT) {
                        const R t = a.cf.s_re[s] * xpr - a.cf.s_im[s] * xpi;
                        xpi = a.cf.s_re[s] * xpi + a.cf.s_im[s] * xpr;
                        xpr = t;
                    }
                    const R dr = xr - xpr, di = xi - xpi;
                    const R qr = rhr - bxr, qi = rhi - bxi;
                    yc[c][2 * v] = xr + (ar * dr - ai * di) + (cr * qr - ci * qi);
                    yc[c][2 * v + 1] = xi + (ar * di + ai * dr) + (cr * qi + ci * qr);
                }
                if (!FINAL && store_ok) stc<R, 2 * VX>(gptr(a.out) + a.soff[s] + 2u * pt, yc[c]);
            } else if (FINAL) {
                const bool rs = (a.src[s] == SRC_RHAT);
                const R sr = rs ? a.cf.s_re[s] : R(1), si = rs ? a.cf.s_im[s] : R(0);
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    yc[c][2 * v] = sr * pc[c][2 * v] - si * pc[c][2 * v + 1];
                    yc[c][2 * v + 1] = sr * pc[c][2 * v + 1] + si * pc[c][2 * v];
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
                    double acc = static_cast<double>(yr[0][v]);
                    if (NSR == 2) acc += ((k & 1) ? -1.0 : 1.0) * static_cast<double>(yr[NSR - 1][v]);
                    double sum = 0.0;
#pragma unroll
                    for (int c = 0; c < NSC; ++c) {
                        const int j = ((c + 1) * k) % ELL;
                        sum += static_cast<double>(yc[c][2 * v]) * a.cw[j] -
                               static_cast<double>(yc[c][2 * v + 1]) * a.sw[j];
                    }
                    zk[v] = a.ginv[k] * (acc + 2.0 * sum);
                }
                stv_nt<double, VX>(gptr(a.z) + static_cast<size_t>(k) * static_cast<size_t>(a.g.n) + pt, zk);
            }
        }
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    load_row(I0{}, y0 - 1);
    load_row(I1{}, y0);
    // rows rotate through the three window slots: (p, c, n) = (0,1,2), (1,2,0), (2,0,1)
    int y = y0;
    while (y < y1) {
        load_row(I2{}, y + 1);
        load_centre(y);
        compute_row(I0{}, I1{}, I2{}, y);
        if (++y >= y1) break;
        load_row(I0{}, y + 1);
        load_centre(y);
        compute_row(I1{}, I2{}, I0{}, y);
        if (++y >= y1) break;
        load_row(I1{}, y + 1);
        load_centre(y);
        compute_row(I2{}, I0{}, I1{}, y);
        ++y;
    }
}

template <typename R, typename KS, int ELL, int VX, bool CUR_RHAT, bool FINAL, bool PER>
__global__ __launch_bounds__(256) void cheb_sweep_kernel(const SweepArgs<R> a) {
    cheb_sweep_body<R, KS, ELL, VX, CUR_RHAT, FINAL, PER>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Forward scaled time-DFT: per grid point, t_k = gam_k r_k and
// rhat_m = sum_k t_k exp(-2 pi i m k / l) for the l_s unique m, in float64,
// stored in the inner real type.  The Krylov input is read and the transforms are
// written with non-temporal accesses (each is touched once here).

// The transform of one lane's VX points from their scaled values t[k][x].
template <typename R, int ELL, int VX>
__device__ __forceinline__ void tdft_fwd_store(const FwdArgs& a, long long i0, const double (&t)[ELL][VX]) {
    constexpr int NSR = (ELL % 2 == 0) ? 2 : 1;
    constexpr int NSC = (ELL - NSR) / 2;
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
        stv_nt<R, VX>(static_cast<R*>(a.rhat[0]) + i0, o0);
        if (NSR == 2) stv_nt<R, VX>(static_cast<R*>(a.rhat[1]) + i0, o1);
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
        stv_nt<R, 2 * VX>(static_cast<R*>(a.rhat[NSR + c]) + 2 * i0, o);
    }
}

template <typename R, int ELL, int VX>
__device__ __forceinline__ void tdft_fwd_body(const FwdArgs& a, int bid, double mul) {
    const long long i0 = (static_cast<long long>(bid) * blockDim.x + threadIdx.x) * VX;
    if (i0 >= a.n) return;
    double t[ELL][VX];
#pragma unroll
    for (int k = 0; k < ELL; ++k) {
        double v[VX];
        ldv_nt<double, VX>(a.r + static_cast<long long>(k) * a.n + i0, v);
        const double gk = a.gam[k] * mul;
#pragma unroll
        for (int x = 0; x < VX; ++x) t[k][x] = gk * v[x];
    }
    tdft_fwd_store<R, ELL, VX>(a, i0, t);
}

// The Gram-Schmidt update of the newest Krylov vector fused with the forward
// transform that starts the next preconditioner application: per grid point and
// block k, w_k <- w_k - sum_{q < nv} c_q V_q,k (written back), t_k = gam_k w_k, and
// the l_s transforms of t; the block's sum of w^2 goes to partial[block * stride].
// The transform is of the new vector as it stands (gam carries no input scale): the
// caller scales the preconditioned result once the norm is known.  A grid-stride
// loop over the points; blocks of 256 threads.
template <typename R, int ELL, int VX, int NVB>
__global__ __launch_bounds__(256) void axpy_fwd_kernel(const AxpyFwdArgs a) {
    const FwdArgs& f = a.f;
    double ssq = 0.0;
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x * VX;
    for (long long i0 = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) * VX; i0 < f.n; i0 += step) {
        double t[ELL][VX];
#pragma unroll
        for (int k = 0; k < ELL; ++k) {
            double* wk = gptr(a.w) + static_cast<long long>(k) * f.n + i0;
            double wv[VX];
            ldv_nt<double, VX>(wk, wv);
#pragma unroll
            for (int q = 0; q < NVB; ++q) {
                if (q < a.nv) {
                    double v[VX];
                    ldv_nt<double, VX>(gptr(a.v[q]) + static_cast<long long>(k) * f.n + i0, v);
#pragma unroll
                    for (int x = 0; x < VX; ++x) wv[x] -= a.c[q] * v[x];
                }
            }
            stv_nt<double, VX>(wk, wv);
#pragma unroll
            for (int x = 0; x < VX; ++x) {
                ssq += wv[x] * wv[x];
                t[k][x] = f.gam[k] * wv[x];
            }
        }
        tdft_fwd_store<R, ELL, VX>(f, i0, t);
    }
    __shared__ double red[4];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) ssq += __shfl_down(ssq, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = ssq;
    __syncthreads();
    if (threadIdx.x == 0) gptr(a.partial)[static_cast<long long>(blockIdx.x) * a.stride] = red[0] + red[1] + red[2] + red[3];
}

template <typename R, int ELL, int VX>
__global__ __launch_bounds__(256) void tdft_fwd_kernel(const FwdArgs a) {
    tdft_fwd_body<R, ELL, VX>(a, blockIdx.x, 1.0);
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
__device__ __forceinline__ void apply_calA_body(const CalAArgs& a, int bid, int nb) {
    const long long tile = tile_of_wave(a.t, bid, nb);
    const int lane = threadIdx.x & (kWave - 1);
    double ssq = 0.0;
    if (tile >= 0) {
        const Geom& g = a.g;
        const double* __restrict__ kappa = gptr(a.kappa);
        const double* __restrict__ ax = gptr(a.x);
        const int sx = static_cast<int>(tile % a.t.nsx);
        const int cy = static_cast<int>(tile / a.t.nsx);
        const int x0 = sx * kWave * VX;
        const int y0 = cy * a.t.h;
        const int y1 = min(y0 + a.t.h, g.ny);

        double kp[VX], kc[VX], kn[VX], khc, khn, kd;
        double xp[ELL][VX], xc[ELL][VX], xn[ELL][VX], hc[ELL], hn[ELL], hd;
        load_real_row<double, VX, double>(kappa, g, y0 - 1, x0, lane, kp, kd);
        load_real_row<double, VX, double>(kappa, g, y0, x0, lane, kc, khc);
#pragma unroll
        for (int k = 0; k < ELL; ++k) {
            load_real_row<double, VX, double>(ax + k * g.n, g, y0 - 1, x0, lane, xp[k], hd);
            load_real_row<double, VX, double>(ax + k * g.n, g, y0, x0, lane, xc[k], hc[k]);
        }
        for (int y = y0; y < y1; ++y) {
            load_real_row<double, VX, double>(kappa, g, y + 1, x0, lane, kn, khn);
#pragma unroll
            for (int k = 0; k < ELL; ++k)
                load_real_row<double, VX, double>(ax + k * g.n, g, y + 1, x0, lane, xn[k], hn[k]);

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
                        ldv<double, VX>(gptr(a.b) + k * g.n + rowoff + xb, bb);
#pragma unroll
                        for (int v = 0; v < VX; ++v) {
                            yo[v] = bb[v] - yo[v];
                            ssq += yo[v] * yo[v];
                        }
                    }
                    stv<double, VX>(gptr(a.y) + k * g.n + rowoff + xb, yo);
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
        if (lane == 0 && tile >= 0) gptr(a.partial)[tile] = ssq;
    }
}

template <int ELL, int VX, bool RESID>
__global__ __launch_bounds__(256) void apply_calA_kernel(const CalAArgs a) {
    apply_calA_body<ELL, VX, RESID>(a, blockIdx.x, gridDim.x);
}

// The same operator on Dirichlet grids without halo loads: a wave loads 64*VX
// consecutive columns starting VX columns left of the 64*VX - 2*VX columns it owns
// (strips overlap by 2*VX columns), so lanes 1..62 own their points and the two edge
// lanes only supply east / west neighbours, which cross lanes by DPP shifts.  Ghost
// rows and columns read zeros through raw buffer loads (a block of N values must fit
// a buffer range, N * 8 < 2^31 bytes).  Against the halo-load form this needs no
// per-lane halo registers (84 against 176 VGPRs at l = 10, one point per lane) and no
// single-lane halo loads.  The result is written with non-temporal stores: the next
// kernel (the multi-dot that reads it, or the next preconditioner stage) then runs
// without the write-back of this kernel's dirty lines, which measured faster over a
// whole solve although this kernel alone is a little slower.
template <int ELL, int VX, bool RESID, bool UP>
__device__ __forceinline__ void apply_calA_strip_rows(const CalAArgs& a, long long tile) {
    constexpr int W = kWave * VX;
    constexpr int S = W - 2 * VX;  // owned columns per strip
    const int lane = threadIdx.x & (kWave - 1);
    double ssq = 0.0;
    if (tile >= 0) {
        const Geom& g = a.g;
        const int nx = g.nx, ny = g.ny;
        const int sx = static_cast<int>(tile % a.t.nsx);
        const int cy = static_cast<int>(tile / a.t.nsx);
        const int xb = sx * S - VX + lane * VX;  // first column of this lane
        const bool colok = xb >= 0 && xb + VX <= nx;
        const bool own = colok && lane > 0 && lane < kWave - 1;
        const int y0 = cy * a.t.h;
        const int y1 = min(y0 + a.t.h, ny);
        const unsigned nb = static_cast<unsigned>(g.n) * 8u;
        const __amdgpu_buffer_rsrc_t rk = buf_rsrc(a.kappa, nb);
        auto load_row = [&](int y, double (&kr)[VX], double (&xr)[ELL][VX]) {
            const unsigned off = (colok && y >= 0 && y < ny) ? static_cast<unsigned>(y * nx + xb) * 8u : kOob;
            bld<0>(rk, off, kr);
#pragma unroll
            for (int k = 0; k < ELL; ++k) bld<0>(buf_rsrc(a.x + static_cast<long long>(k) * g.n, nb), off, xr[k]);
        };
        // p: the row behind the march, n: the row ahead (UP: rows y + 1 and y - 1)
        constexpr int dy = UP ? -1 : 1;
        double kp[VX], kc[VX], kn[VX];
        double xp[ELL][VX], xc[ELL][VX], xn[ELL][VX];
        const int ys = UP ? y1 - 1 : y0;
        load_row(ys - dy, kp, xp);
        load_row(ys, kc, xc);
        for (int i = 0, y = ys; i < y1 - y0; ++i, y += dy) {
            load_row(y + dy, kn, xn);
            const double (&ks)[VX] = UP ? kn : kp;  // south (y - 1) and north (y + 1) rows
            const double (&kq)[VX] = UP ? kp : kn;
            const double (&xs)[ELL][VX] = UP ? xn : xp;
            const double (&xq)[ELL][VX] = UP ? xp : xn;
            const long long ro = static_cast<long long>(y) * nx + xb;
            const double kwv = from_west0(kc[VX - 1]);
            const double kev = from_east0(kc[0]);
            Faces<double> fc[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const double kw = (v > 0) ? kc[v - 1] : kwv;
                const double ke = (v < VX - 1) ? kc[v + 1] : kev;
                fc[v] = faces<double>(g, xb + v, y, kc[v], kw, ke, ks[v], kq[v]);
            }
#pragma unroll
            for (int k = 0; k < ELL; ++k) {
                const double wv = from_west0(xc[k][VX - 1]);
                const double ev = from_east0(xc[k][0]);
                double yo[VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const double xw = (v > 0) ? xc[k][v - 1] : wv;
                    const double xe = (v < VX - 1) ? xc[k][v + 1] : ev;
                    double ax = fc[v].diag * xc[k][v];
                    ax -= fc[v].w * xw + fc[v].e * xe + fc[v].s * xs[k][v] + fc[v].n * xq[k][v];
                    if (k > 0) ax -= xc[k - 1][v];
                    yo[v] = ax;
                }
                if (own) {
                    if (RESID) {
                        double bb[VX];
                        ldv_nt<double, VX>(gptr(a.b) + k * g.n + ro, bb);
#pragma unroll
                        for (int v = 0; v < VX; ++v) {
                            yo[v] = bb[v] - yo[v];
                            ssq += yo[v] * yo[v];
                        }
                    }
                    stv_nt<double, VX>(gptr(a.y) + k * g.n + ro, yo);
                }
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                kp[v] = kc[v];
                kc[v] = kn[v];
            }
#pragma unroll
            for (int k = 0; k < ELL; ++k) {
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    xp[k][v] = xc[k][v];
                    xc[k][v] = xn[k][v];
                }
            }
        }
    }
    if (RESID) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) ssq += __shfl_down(ssq, off, kWave);
        if (lane == 0 && tile >= 0) gptr(a.partial)[tile] = ssq;
    }
}

// Chunks march down on even chunk rows and up on odd ones, so two neighbouring chunks
// reach the rows they share (each one's halo row is the other's edge row) at about the
// same time, and the second read of those rows can hit the cache.
template <int ELL, int VX, bool RESID>
__device__ __forceinline__ void apply_calA_strip_body(const CalAArgs& a, long long tile) {
    if (tile >= 0 && ((tile / a.t.nsx) & 1)) apply_calA_strip_rows<ELL, VX, RESID, true>(a, tile);
    else apply_calA_strip_rows<ELL, VX, RESID, false>(a, tile);
}

template <int ELL, int VX, bool RESID>
__global__ __launch_bounds__(256) void apply_calA_strip_kernel(const CalAArgs a) {
    apply_calA_strip_body<ELL, VX, RESID>(a, tile_of_wave(a.t, blockIdx.x, gridDim.x));
}

// Varying diagonal blocks: y_k = A_k x_k - x_{k-1} with A_k built from the block's own
// coefficient field kappa + k*N.  One wave per (tile, block k = blockIdx.y); x_{k-1}
// enters only through its centre row.  Residual mode as above, partial index
// k * tiles + tile.
template <int VX, bool RESID>
__global__ __launch_bounds__(256) void apply_calA_var_kernel(const CalAArgs a) {
    const int k = blockIdx.y;
    const long long tile = tile_of_wave(a.t, blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & (kWave - 1);
    double ssq = 0.0;
    if (tile >= 0) {
        const Geom& g = a.g;
        const int sx = static_cast<int>(tile % a.t.nsx);
        const int cy = static_cast<int>(tile / a.t.nsx);
        const int x0 = sx * kWave * VX;
        const int y0 = cy * a.t.h;
        const int y1 = min(y0 + a.t.h, g.ny);
        const double* kap = a.kappa + static_cast<long long>(k) * g.n;
        const double* xk = a.x + static_cast<long long>(k) * g.n;
        double kp[VX], kc[VX], kn[VX], khc, khn, kd;
        double xp[VX], xc[VX], xn[VX], hc, hn, hd;
        load_real_row<double, VX, double>(kap, g, y0 - 1, x0, lane, kp, kd);
        load_real_row<double, VX, double>(kap, g, y0, x0, lane, kc, khc);
        load_real_row<double, VX, double>(xk, g, y0 - 1, x0, lane, xp, hd);
        load_real_row<double, VX, double>(xk, g, y0, x0, lane, xc, hc);
        const int xb = x0 + lane * VX;
        const bool store_ok = xb < g.nx;
        for (int y = y0; y < y1; ++y) {
            load_real_row<double, VX, double>(kap, g, y + 1, x0, lane, kn, khn);
            load_real_row<double, VX, double>(xk, g, y + 1, x0, lane, xn, hn);
            const long long rowoff = static_cast<long long>(y) * g.nx;
            double xprev[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) xprev[v] = 0.0;
            if (k > 0 && store_ok) ldv<double, VX>(a.x + static_cast<long long>(k - 1) * g.n + rowoff + xb, xprev);
            const double kwv = shfl_up1(kc[VX - 1]);
            const double kev = shfl_dn1(kc[0]);
            const double wv = shfl_up1(xc[VX - 1]);
            const double ev = shfl_dn1(xc[0]);
            double yo[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const double kw = (v > 0) ? kc[v - 1] : (lane == 0 ? khc : kwv);
                const double ke = (v < VX - 1) ? kc[v + 1] : (lane == kWave - 1 ? khc : kev);
                const Faces<double> f = faces<double>(g, xb + v, y, kc[v], kw, ke, kp[v], kn[v]);
                const double xw = (v > 0) ? xc[v - 1] : (lane == 0 ? hc : wv);
                const double xe = (v < VX - 1) ? xc[v + 1] : (lane == kWave - 1 ? hc : ev);
                double ax = f.diag * xc[v];
                ax -= f.w * xw + f.e * xe + f.s * xp[v] + f.n * xn[v];
                yo[v] = ax - xprev[v];
            }
            if (store_ok) {
                if (RESID) {
                    double bb[VX];
                    ldv<double, VX>(a.b + static_cast<long long>(k) * g.n + rowoff + xb, bb);
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        yo[v] = bb[v] - yo[v];
                        ssq += yo[v] * yo[v];
                    }
                }
                stv<double, VX>(a.y + static_cast<long long>(k) * g.n + rowoff + xb, yo);
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                kp[v] = kc[v];
                kc[v] = kn[v];
                xp[v] = xc[v];
                xc[v] = xn[v];
            }
            khc = khn;
            hc = hn;
        }
    }
    if (RESID) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) ssq += __shfl_down(ssq, off, kWave);
        if (lane == 0 && tile >= 0) a.partial[static_cast<long long>(k) * a.t.tiles + tile] = ssq;
    }
}

// ---------------------------------------------------------------------------
// Batched launches over a work list of independent problems (uneven grids): member q
// has its arguments in args[q] and first[q + 1] - first[q] blocks of its own launch;
// members whose problem is not live (convergence mask) get no blocks (worklist.h).

__device__ __forceinline__ LiveBlocks list_live_blocks(const BatchList& L) {
    return live_blocks(
        L.nprob, [&](int q) { return L.first[q + 1] - L.first[q]; }, [&](int q) { return L.live[L.pid[q]] != 0; });
}

template <typename R, typename KS, int ELL, int VX, bool CUR_RHAT, bool FINAL>
__global__ __launch_bounds__(256) void cheb_sweep_batch_kernel(const BatchList L) {
    const LiveBlocks W = list_live_blocks(L);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const SweepArgs<R>& a = list_args<SweepArgs<R>>(L.args, q);
        cheb_sweep_body<R, KS, ELL, VX, CUR_RHAT, FINAL, false>(a, local, nb);
    }
}

template <typename R, int ELL, int VX>
__global__ __launch_bounds__(256) void tdft_fwd_batch_kernel(const BatchList L) {
    const LiveBlocks W = list_live_blocks(L);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const FwdArgs& a = list_args<FwdArgs>(L.args, q);
        tdft_fwd_body<R, ELL, VX>(a, local, L.scale ? L.scale[L.pid[q]] : 1.0);
    }
}

template <int ELL, int VX, bool RESID, bool STRIPS>
__global__ __launch_bounds__(256) void apply_calA_batch_kernel(const BatchList L) {
    const LiveBlocks W = list_live_blocks(L);
    for (int v = blockIdx.x; v < W.total; v += gridDim.x) {
        int q, local, nb;
        if (!live_block(W, v, q, local, nb)) continue;
        const CalAArgs& a = list_args<CalAArgs>(L.args, q);
        if (STRIPS) apply_calA_strip_body<ELL, VX, RESID>(a, tile_of_wave(a.t, local, nb));
        else apply_calA_body<ELL, VX, RESID>(a, local, nb);
    }
}

}  // namespace
}  // namespace ac
