// Inner solves of the saddle-point preconditioner P_SP (Section 4).
//
// A complex shifted system (A - lambda I) x = b, lambda = rho + i s, is solved in real
// arithmetic as the saddle system of eq. (saddlesystem),
//   [[sigma I, A - rho I], [A - rho I, -sigma I]] u = f,  sigma = |s|,
// with u = (Re x, -Im x), f = (-Im b, Re b) for s > 0 and u = (Re x, Im x),
// f = (Im b, Re b) for s < 0, by preconditioned MINRES with P_D = blkdiag(A - (rho -
// sigma) I) twice (eq. (minresprecond)) applied by V-cycles; a real shift by
// preconditioned CG with a V-cycle for A - lambda I (Section 5).  Every shift runs the
// same number of iterations from a zero guess, all in lockstep so that one batched
// V-cycle serves every shift.  The MINRES and CG scalars live on the device (a
// single-block kernel updates them from the reduced inner products), so an application
// needs no host synchronisation.  Vectors are float64, or float32 with the multigrid's
// float32 coefficient copies (the inner products and the scalars stay float64).
//
// MINRES (Paige-Saunders, Lanczos form with an SPD preconditioner): from v_1 = f,
// z_1 = M^{-1} v_1, gamma_1 = sqrt(v_1 . z_1), eta = gamma_1, c_0 = c_1 = 1,
// s_0 = s_1 = 0, w_0 = w_1 = 0, each step: z_j /= gamma_j; delta = (S z_j) . z_j;
// v_{j+1} = S z_j - (delta/gamma_j) v_j - (gamma_j/gamma_{j-1}) v_{j-1};
// z_{j+1} = M^{-1} v_{j+1}; gamma_{j+1} = sqrt(v_{j+1} . z_{j+1}); the Givens rotation
// a0 = c_j delta - c_{j-1} s_j gamma_j, a1 = hypot(a0, gamma_{j+1}),
// a2 = s_j delta + c_{j-1} c_j gamma_j, a3 = s_{j-1} gamma_j, c_{j+1} = a0/a1,
// s_{j+1} = gamma_{j+1}/a1; w_{j+1} = (z_j - a3 w_{j-1} - a2 w_j)/a1;
// x += c_{j+1} eta w_{j+1}; eta = -s_{j+1} eta.  A step that finds gamma_{j+1} = 0 (the
// exact solution) is the last one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr int kBlk = 2048;  // blocks of the reducing kernels (grid-stride)
constexpr int kThr = 256;
constexpr int kSt = 16;     // state doubles per shift

// complex-slot state
enum { G = 0, GP, ETA, C, CP, S, SP, DONE, A1, A2, A3, XC, GINV, SKIP };
// real-slot state
enum { RHO = 0, RDONE = 1, ALPHA = 2, BETA = 3 };

template <typename T>
struct Vec9 {
    T* p[kMaxShift];
};
template <typename T>
struct CVec9 {
    const T* p[kMaxShift];
};

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kThr / kWave];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThr / kWave; ++w) t += red[w];
    return t;
}

// Coefficients of the fine level at point i (float64 arithmetic on the stored type: the
// float64 arrays, or their float32 copies for float32 vectors); a missing neighbour has
// coefficient 0 and its value is not read.
struct Fine {
    double d, e, w, n, s;
    bool he, hw, hn, hs;
    long long nx;
};
template <typename T>
__device__ __forceinline__ Fine fine_at(const MgLevel& L, long long i) {
    const int ii = static_cast<int>(i), x = ii % L.nx, y = ii / L.nx;
    Fine f;
    f.nx = L.nx;
    f.he = x < L.nx - 1;
    f.hw = x > 0;
    f.hn = L.dim == 2 && y < L.ny - 1;
    f.hs = L.dim == 2 && y > 0;
    if constexpr (std::is_same<T, float>::value) {
        f.d = L.diag_f[i];
        f.e = f.he ? L.wx_f[i] : 0.0;
        f.w = f.hw ? L.wx_f[i - 1] : 0.0;
        f.n = f.hn ? L.wy_f[i] : 0.0;
        f.s = f.hs ? L.wy_f[i - L.nx] : 0.0;
    } else {
        f.d = L.diag[i];
        f.e = f.he ? L.wx[i] : 0.0;
        f.w = f.hw ? L.wx[i - 1] : 0.0;
        f.n = f.hn ? L.wy[i] : 0.0;
        f.s = f.hs ? L.wy[i - L.nx] : 0.0;
    }
    return f;
}
// (A - c I) u at point i
template <typename T>
__device__ __forceinline__ double op_at(const Fine& f, const T* __restrict__ u, long long i, double c) {
    double a = (f.d - c) * static_cast<double>(u[i]);
    if (f.he) a -= f.e * static_cast<double>(u[i + 1]);
    if (f.hw) a -= f.w * static_cast<double>(u[i - 1]);
    if (f.hn) a -= f.n * static_cast<double>(u[i + f.nx]);
    if (f.hs) a -= f.s * static_cast<double>(u[i - f.nx]);
    return a;
}

// Sz = S (z / gamma) per complex slot (blockIdx.y), partial[blk * ns + q] of
// (S z/gamma) . (z/gamma).  A finished slot writes zeros.
template <typename T>
__global__ __launch_bounds__(kThr) void saddle_apply_kernel(const MgLevel L, long long n, CVec9<T> z, Vec9<T> sz,
                                                            const double* __restrict__ st, SpProblem P,
                                                            double* __restrict__ partial, int ns) {
    const int q = blockIdx.y;
    const double* sq = st + q * kSt;
    const bool done = sq[DONE] != 0.0;
    const double ginv = done ? 0.0 : 1.0 / sq[G];
    const double sig = P.sigma[q], rho = P.rho[q];
    const T* __restrict__ z1 = z.p[q];
    const T* __restrict__ z2 = z1 + n;
    T* __restrict__ o1 = sz.p[q];
    T* __restrict__ o2 = o1 + n;
    double acc = 0.0;
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * kThr) {
        if (done) {
            o1[i] = T(0);
            o2[i] = T(0);
            continue;
        }
        const Fine f = fine_at<T>(L, i);
        const double a1 = z1[i], a2 = z2[i];
        const double t1 = (sig * a1 + op_at(f, z2, i, rho)) * ginv;
        const double t2 = (op_at(f, z1, i, rho) - sig * a2) * ginv;
        o1[i] = static_cast<T>(t1);
        o2[i] = static_cast<T>(t2);
        acc += (t1 * a1 + t2 * a2) * ginv;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[static_cast<long long>(blockIdx.x) * ns + q] = t;
}

// VX consecutive points of one grid row per thread (nx % VX == 0, so a vector never
// crosses a row): vector loads of the centre values and of the rows above and below,
// clamped addresses for neighbours past the grid (their coefficients are zero there, so
// they subtract nothing), no branch around a load.  The memory instructions per point
// drop about VX-fold; the arithmetic per point is op_at's, term for term.
template <typename T, int V>
__device__ __forceinline__ void ldvec(const T* p, T (&o)[V]) {
    typedef T TV __attribute__((ext_vector_type(V)));
    const TV t = *reinterpret_cast<const TV*>(p);
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = t[v];
}
template <typename T, int V>
__device__ __forceinline__ void stvec(T* p, const T (&in)[V]) {
    typedef T TV __attribute__((ext_vector_type(V)));
    TV t;
#pragma unroll
    for (int v = 0; v < V; ++v) t[v] = in[v];
    *reinterpret_cast<TV*>(p) = t;
}

template <int VX>
struct FineV {
    double d[VX], e[VX], w[VX], n[VX], s[VX];
    int x0;
    bool hn, hs;
};
template <typename T, int VX>
__device__ __forceinline__ FineV<VX> fine_v(const MgLevel& L, long long i0) {
    const int ii = static_cast<int>(i0), x0 = ii % L.nx, y = ii / L.nx;
    const long long nx = L.nx;
    FineV<VX> f;
    f.x0 = x0;
    f.hn = L.dim == 2 && y < L.ny - 1;
    f.hs = L.dim == 2 && y > 0;
    T dv[VX], wxv[VX], wyn[VX], wys[VX];
    const T* __restrict__ dg = std::is_same<T, float>::value ? reinterpret_cast<const T*>(L.diag_f)
                                                             : reinterpret_cast<const T*>(L.diag);
    const T* __restrict__ wx = std::is_same<T, float>::value ? reinterpret_cast<const T*>(L.wx_f)
                                                             : reinterpret_cast<const T*>(L.wx);
    const T* __restrict__ wy = std::is_same<T, float>::value ? reinterpret_cast<const T*>(L.wy_f)
                                                             : reinterpret_cast<const T*>(L.wy);
    ldvec<T, VX>(dg + i0, dv);
    ldvec<T, VX>(wx + i0, wxv);
    ldvec<T, VX>(wy + i0, wyn);
    ldvec<T, VX>(wy + (f.hs ? i0 - nx : i0), wys);
    const T wxw = wx[x0 > 0 ? i0 - 1 : i0];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        f.d[v] = dv[v];
        f.e[v] = (x0 + v < L.nx - 1) ? static_cast<double>(wxv[v]) : 0.0;
        f.w[v] = (x0 + v > 0) ? static_cast<double>(v > 0 ? wxv[v - 1] : wxw) : 0.0;
        f.n[v] = f.hn ? static_cast<double>(wyn[v]) : 0.0;
        f.s[v] = f.hs ? static_cast<double>(wys[v]) : 0.0;
    }
    return f;
}
template <typename T, int VX>
__device__ __forceinline__ void op_v(const FineV<VX>& f, const T* __restrict__ u, long long i0, long long nx, int gnx,
                                     double c, double (&out)[VX]) {
    T uc[VX], un[VX], us[VX];
    ldvec<T, VX>(u + i0, uc);
    ldvec<T, VX>(u + (f.hn ? i0 + nx : i0), un);
    ldvec<T, VX>(u + (f.hs ? i0 - nx : i0), us);
    const T uwe = u[f.x0 > 0 ? i0 - 1 : i0];
    const T uee = u[f.x0 + VX < gnx ? i0 + VX : i0];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const T ue = v < VX - 1 ? uc[v + 1] : uee;
        const T uw = v > 0 ? uc[v - 1] : uwe;
        double a = (f.d[v] - c) * static_cast<double>(uc[v]);
        a -= f.e[v] * static_cast<double>(ue);
        a -= f.w[v] * static_cast<double>(uw);
        a -= f.n[v] * static_cast<double>(un[v]);
        a -= f.s[v] * static_cast<double>(us[v]);
        out[v] = a;
    }
}

template <typename T, int VX>
__global__ __launch_bounds__(kThr) void saddle_apply_v_kernel(const MgLevel L, long long n, CVec9<T> z, Vec9<T> sz,
                                                              const double* __restrict__ st, SpProblem P,
                                                              double* __restrict__ partial, int ns) {
    const int q = blockIdx.y;
    const double* sq = st + q * kSt;
    const bool done = sq[DONE] != 0.0;
    const double ginv = done ? 0.0 : 1.0 / sq[G];
    const double sig = P.sigma[q], rho = P.rho[q];
    const T* __restrict__ z1 = z.p[q];
    const T* __restrict__ z2 = z1 + n;
    T* __restrict__ o1 = sz.p[q];
    T* __restrict__ o2 = o1 + n;
    const long long nx = L.nx;
    double acc = 0.0;
    for (long long i0 = (static_cast<long long>(blockIdx.x) * kThr + threadIdx.x) * VX; i0 < n;
         i0 += static_cast<long long>(gridDim.x) * kThr * VX) {
        T r1[VX], r2[VX];
        if (done) {
#pragma unroll
            for (int v = 0; v < VX; ++v) r1[v] = r2[v] = T(0);
            stvec<T, VX>(o1 + i0, r1);
            stvec<T, VX>(o2 + i0, r2);
            continue;
        }
        const FineV<VX> f = fine_v<T, VX>(L, i0);
        T a1v[VX], a2v[VX];
        ldvec<T, VX>(z1 + i0, a1v);
        ldvec<T, VX>(z2 + i0, a2v);
        double op1[VX], op2[VX];
        op_v<T, VX>(f, z2, i0, nx, L.nx, rho, op2);
        op_v<T, VX>(f, z1, i0, nx, L.nx, rho, op1);
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const double a1 = a1v[v], a2 = a2v[v];
            const double t1 = (sig * a1 + op2[v]) * ginv;
            const double t2 = (op1[v] - sig * a2) * ginv;
            r1[v] = static_cast<T>(t1);
            r2[v] = static_cast<T>(t2);
            acc += (t1 * a1 + t2 * a2) * ginv;
        }
        stvec<T, VX>(o1 + i0, r1);
        stvec<T, VX>(o2 + i0, r2);
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[static_cast<long long>(blockIdx.x) * ns + q] = t;
}

template <typename T, int VX>
__global__ __launch_bounds__(kThr) void cg_apply_v_kernel(const MgLevel L, long long n, CVec9<T> pv, Vec9<T> qv,
                                                          SpProblem P, double* __restrict__ partial, int ns) {
    const int r = blockIdx.y;
    const T* __restrict__ p = pv.p[r];
    T* __restrict__ q = qv.p[r];
    const long long nx = L.nx;
    double acc = 0.0;
    for (long long i0 = (static_cast<long long>(blockIdx.x) * kThr + threadIdx.x) * VX; i0 < n;
         i0 += static_cast<long long>(gridDim.x) * kThr * VX) {
        double a[VX];
        op_v<T, VX>(fine_v<T, VX>(L, i0), p, i0, nx, L.nx, P.lam[r], a);
        T pc[VX], qo[VX];
        ldvec<T, VX>(p + i0, pc);
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            qo[v] = static_cast<T>(a[v]);
            acc += static_cast<double>(pc[v]) * a[v];
        }
        stvec<T, VX>(q + i0, qo);
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[static_cast<long long>(blockIdx.x) * ns + P.nc + r] = t;
}

// q = (A - lambda I) p per real slot, partial of p . q (slot index nc + r)
template <typename T>
__global__ __launch_bounds__(kThr) void cg_apply_kernel(const MgLevel L, long long n, CVec9<T> pv, Vec9<T> qv,
                                                        SpProblem P, double* __restrict__ partial, int ns) {
    const int r = blockIdx.y;
    const T* __restrict__ p = pv.p[r];
    T* __restrict__ q = qv.p[r];
    double acc = 0.0;
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * kThr) {
        const double a = op_at(fine_at<T>(L, i), p, i, P.lam[r]);
        q[i] = static_cast<T>(a);
        acc += static_cast<double>(p[i]) * a;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[static_cast<long long>(blockIdx.x) * ns + P.nc + r] = t;
}

// v_{j+1} = Sz - (delta/gamma) v - (gamma/gamma_prev) v_prev, written over v_prev
template <typename T>
__global__ __launch_bounds__(kThr) void lanczos_kernel(long long len, CVec9<T> sz, CVec9<T> v, Vec9<T> vp,
                                                       const double* __restrict__ st, const double* __restrict__ sums) {
    const int q = blockIdx.y;
    const double* sq = st + q * kSt;
    if (sq[DONE] != 0.0) return;
    const double a = sums[q] / sq[G], b = sq[G] / sq[GP];
    const T* __restrict__ s = sz.p[q];
    const T* __restrict__ vv = v.p[q];
    T* __restrict__ o = vp.p[q];
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < len;
         i += static_cast<long long>(gridDim.x) * kThr)
        o[i] = static_cast<T>(static_cast<double>(s[i]) - a * static_cast<double>(vv[i]) - b * static_cast<double>(o[i]));
}

// CG: x += a p, r -= a q with a = rho / (p . q)
template <typename T>
__global__ __launch_bounds__(kThr) void cg_update1_kernel(long long n, CVec9<T> pv, CVec9<T> qv, Vec9<T> xv,
                                                          Vec9<T> rv, const double* __restrict__ st,
                                                          const double* __restrict__ sums, int nc) {
    const int r = blockIdx.y;
    const double* sr = st + (nc + r) * kSt;
    if (sr[RDONE] != 0.0) return;
    const double a = sr[RHO] / sums[nc + r];
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * kThr) {
        xv.p[r][i] = static_cast<T>(static_cast<double>(xv.p[r][i]) + a * static_cast<double>(pv.p[r][i]));
        rv.p[r][i] = static_cast<T>(static_cast<double>(rv.p[r][i]) - a * static_cast<double>(qv.p[r][i]));
    }
}

// partial[blk * ns + k] of a_k . b_k over len_k entries
template <typename T>
struct DotArgs {
    const T* a[2 * kMaxShift];
    const T* b[2 * kMaxShift];
    long long len[2 * kMaxShift];
};
template <typename T>
__global__ __launch_bounds__(kThr) void dot_kernel(DotArgs<T> d, double* __restrict__ partial, int ns) {
    const int k = blockIdx.y;
    const T* __restrict__ a = d.a[k];
    const T* __restrict__ b = d.b[k];
    double acc = 0.0;
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < d.len[k];
         i += static_cast<long long>(gridDim.x) * kThr)
        acc += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[static_cast<long long>(blockIdx.x) * ns + k] = t;
}
// Scalars after the preconditioner step (one thread per slot).  init: start values from
// gamma_1^2 / rho_0 in sums; else the MINRES rotation (sumsA: delta, sumsB: gamma_{j+1}^2)
// and the CG beta.
__global__ void coef_kernel(double* __restrict__ st, const double* __restrict__ sumsA,
                            const double* __restrict__ sumsB, int nc, int nr, int init) {
    const int q = threadIdx.x;
    if (q < nc) {
        double* s = st + q * kSt;
        if (init) {
            const double g = sqrt(fmax(sumsB[q], 0.0));
            s[G] = g;
            s[GP] = 1.0;
            s[ETA] = g;
            s[C] = s[CP] = 1.0;
            s[S] = s[SP] = 0.0;
            s[DONE] = g == 0.0 ? 1.0 : 0.0;
            s[SKIP] = s[DONE];
            return;
        }
        s[SKIP] = s[DONE];
        if (s[DONE] != 0.0) return;
        const double delta = sumsA[q], g = s[G];
        const double gn = sqrt(fmax(sumsB[q], 0.0));
        const double a0 = s[C] * delta - s[CP] * s[S] * g;
        const double a1 = hypot(a0, gn);
        const double a2 = s[S] * delta + s[CP] * s[C] * g;
        const double a3 = s[SP] * g;
        const double cn = a0 / a1, sn = gn / a1;
        s[CP] = s[C];
        s[C] = cn;
        s[SP] = s[S];
        s[S] = sn;
        s[A1] = a1;
        s[A2] = a2;
        s[A3] = a3;
        s[XC] = cn * s[ETA];
        s[GINV] = 1.0 / g;
        s[ETA] = -sn * s[ETA];
        s[GP] = g;
        s[G] = gn;
        if (gn == 0.0) s[DONE] = 1.0;
    } else if (q < nc + nr) {
        double* s = st + q * kSt;
        const double rn = sumsB[q];
        if (init) {
            s[RHO] = rn;
            s[RDONE] = rn == 0.0 ? 1.0 : 0.0;
            s[BETA] = 0.0;
            return;
        }
        if (s[RDONE] != 0.0) {
            s[BETA] = 0.0;
            return;
        }
        s[BETA] = rn / s[RHO];
        s[RHO] = rn;
        if (rn == 0.0) s[RDONE] = 1.0;
    }
}

// w_{j+1} = (z_j / gamma_j - a3 w_{j-1} - a2 w_j) / a1 over w_{j-1}; x += c eta w_{j+1}
template <typename T>
__global__ __launch_bounds__(kThr) void minres_update_kernel(long long len, CVec9<T> z, CVec9<T> w, Vec9<T> wp,
                                                             Vec9<T> x, const double* __restrict__ st) {
    const int q = blockIdx.y;
    const double* s = st + q * kSt;
    if (s[SKIP] != 0.0) return;
    const double gi = s[GINV], a1 = s[A1], a2 = s[A2], a3 = s[A3], xc = s[XC];
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < len;
         i += static_cast<long long>(gridDim.x) * kThr) {
        const double wn = (static_cast<double>(z.p[q][i]) * gi - a3 * static_cast<double>(wp.p[q][i]) -
                           a2 * static_cast<double>(w.p[q][i])) / a1;
        wp.p[q][i] = static_cast<T>(wn);
        x.p[q][i] = static_cast<T>(static_cast<double>(x.p[q][i]) + xc * wn);
    }
}

// CG: p = z + beta p (init: p = z)
template <typename T>
__global__ __launch_bounds__(kThr) void cg_update2_kernel(long long n, CVec9<T> z, Vec9<T> p,
                                                          const double* __restrict__ st, int nc, int init) {
    const int r = blockIdx.y;
    const double* s = st + (nc + r) * kSt;
    if (!init && s[RDONE] != 0.0 && s[BETA] == 0.0) return;
    const double b = init ? 0.0 : s[BETA];
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * kThr)
        p.p[r][i] = init ? z.p[r][i]
                         : static_cast<T>(static_cast<double>(z.p[r][i]) + b * static_cast<double>(p.p[r][i]));
}

// Start vectors: complex slots f from the interleaved right-hand side, zero v_prev, w, w_prev
// and x; real slots r = b, x = 0.  blockIdx.y = slot (complex first).
template <typename T>
struct InitArgs {
    CVec9<T> bc, br;
    Vec9<T> v, vp, w, wp, xc, r, xr;
};
template <typename T>
__global__ __launch_bounds__(kThr) void init_kernel(long long n, InitArgs<T> a, SpProblem P) {
    const int q = blockIdx.y;
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * kThr) {
        if (q < P.nc) {
            const T br = a.bc.p[q][2 * i], bi = a.bc.p[q][2 * i + 1];
            a.v.p[q][i] = P.im_pos[q] ? -bi : bi;
            a.v.p[q][n + i] = br;
            a.vp.p[q][i] = a.vp.p[q][n + i] = T(0);
            a.w.p[q][i] = a.w.p[q][n + i] = T(0);
            a.wp.p[q][i] = a.wp.p[q][n + i] = T(0);
            a.xc.p[q][i] = a.xc.p[q][n + i] = T(0);
        } else {
            const int r = q - P.nc;
            a.r.p[r][i] = a.br.p[r][i];
            a.xr.p[r][i] = T(0);
        }
    }
}

// Solutions back to the spectral slots: x = u1 -+ i u2 (complex), x (real)
template <typename T>
__global__ __launch_bounds__(kThr) void final_kernel(long long n, CVec9<T> xc, CVec9<T> xr, SpProblem P) {
    const int q = blockIdx.y;
    for (long long i = static_cast<long long>(blockIdx.x) * kThr + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * kThr) {
        if (q < P.nc) {
            const T u1 = xc.p[q][i], u2 = xc.p[q][n + i];
            T* y = static_cast<T*>(P.yc[q]);
            y[2 * i] = u1;
            y[2 * i + 1] = P.im_pos[q] ? -u2 : u2;
        } else {
            const int r = q - P.nc;
            static_cast<T*>(P.yr[r])[i] = xr.p[r][i];
        }
    }
}

size_t al(size_t d) { return (d + 63) / 64 * 64; }  // elements: 256-byte multiples for either type

template <typename T>
size_t ws_bytes_t(const MgHierarchy& h, long long n, int nc, int nr) {
    const int ns = nc + nr;
    size_t e = 0;
    e += static_cast<size_t>(nc) * 8 * al(2 * n);  // z_a, z_b, Sz, v_prev, v, w_prev, w, x
    e += static_cast<size_t>(nr) * 5 * al(n);      // x, r, z, p, q
    e += al(mg_scratch_elems(h, 2 * nc + nr));
    const size_t d = 2 * al(static_cast<size_t>(kBlk) * ns) + 2 * al(ns) + al(static_cast<size_t>(kSt) * ns);
    return e * sizeof(T) + d * sizeof(double);
}

template <typename T>
hipError_t solve_t(const SpProblem& P, int iters, char* ws, hipStream_t s) {
    const int nc = P.nc, nr = P.nr, ns = nc + nr;
    const long long n = P.n;
    if (ns < 1 || ns > kMaxShift || 2 * nc + nr > kMgMaxVec) return hipErrorInvalidValue;
    double* dp = reinterpret_cast<double*>(ws);
    double* partA = dp;
    dp += al(static_cast<size_t>(kBlk) * ns);
    double* partB = dp;
    dp += al(static_cast<size_t>(kBlk) * ns);
    double* sumsA = dp;
    dp += al(ns);
    double* sumsB = dp;
    dp += al(ns);
    double* st = dp;
    dp += al(static_cast<size_t>(kSt) * ns);
    T* p = reinterpret_cast<T*>(dp);
    auto take = [&](size_t d) {
        T* r = p;
        p += al(d);
        return r;
    };
    T *za[kMaxShift], *zb[kMaxShift], *szb[kMaxShift], *vpb[kMaxShift], *vb[kMaxShift], *wpb[kMaxShift],
        *wb[kMaxShift], *xcb[kMaxShift];
    for (int q = 0; q < nc; ++q) {
        za[q] = take(2 * n);
        zb[q] = take(2 * n);
        szb[q] = take(2 * n);
        vpb[q] = take(2 * n);
        vb[q] = take(2 * n);
        wpb[q] = take(2 * n);
        wb[q] = take(2 * n);
        xcb[q] = take(2 * n);
    }
    T *xr[kMaxShift], *rr[kMaxShift], *zr[kMaxShift], *pr[kMaxShift], *qr[kMaxShift];
    for (int r = 0; r < nr; ++r) {
        xr[r] = take(n);
        rr[r] = take(n);
        zr[r] = take(n);
        pr[r] = take(n);
        qr[r] = take(n);
    }
    T* mgs = take(mg_scratch_elems(*P.h, 2 * nc + nr));
    const MgLevel& L0 = P.h->lev[0];
    const int nb = static_cast<int>(std::min<long long>(kBlk, (2 * n + kThr - 1) / kThr));

    auto cv = [&](T* const* a, int cnt) {
        CVec9<T> v{};
        for (int i = 0; i < cnt; ++i) v.p[i] = a[i];
        return v;
    };
    auto mv = [&](T* const* a, int cnt) {
        Vec9<T> v{};
        for (int i = 0; i < cnt; ++i) v.p[i] = a[i];
        return v;
    };
    // V-cycles: complex halves of src_c (2 each, shift rho - sigma) then real src_r
    auto vcycle = [&](T* const* src_c, T* const* dst_c, T* const* src_r, T* const* dst_r) {
        const T* b[kMgMaxVec];
        T* u[kMgMaxVec];
        double c[kMgMaxVec];
        int k = 0;
        for (int q = 0; q < nc; ++q)
            for (int h = 0; h < 2; ++h) {
                b[k] = src_c[q] + h * n;
                u[k] = dst_c[q] + h * n;
                c[k++] = P.rho[q] - P.sigma[q];
            }
        for (int r = 0; r < nr; ++r) {
            b[k] = src_r[r];
            u[k] = dst_r[r];
            c[k++] = P.lam[r];
        }
        return mg_vcycle(*P.h, k, b, u, c, mgs, s);
    };
    // dots: complex v . z (2n), real r . z (n) -> sumsB
    auto dots = [&](T* const* vc, T* const* zc) -> hipError_t {
        DotArgs<T> d{};
        for (int q = 0; q < nc; ++q) {
            d.a[q] = vc[q];
            d.b[q] = zc[q];
            d.len[q] = 2 * n;
        }
        for (int r = 0; r < nr; ++r) {
            d.a[nc + r] = rr[r];
            d.b[nc + r] = zr[r];
            d.len[nc + r] = n;
        }
        hipLaunchKernelGGL(dot_kernel<T>, dim3(nb, ns), dim3(kThr), 0, s, d, partB, ns);
        return launch_reduce(partB, nb, ns, ns, sumsB, s);
    };

    // start: v_1 = f, z_1 = M^{-1} v_1, gamma_1; r_0 = b, z_0, p_0 = z_0, rho_0
    {
        InitArgs<T> a{};
        for (int q = 0; q < nc; ++q) {
            a.bc.p[q] = static_cast<const T*>(P.bc[q]);
            a.v.p[q] = vb[q];
            a.vp.p[q] = vpb[q];
            a.w.p[q] = wb[q];
            a.wp.p[q] = wpb[q];
            a.xc.p[q] = xcb[q];
        }
        for (int r = 0; r < nr; ++r) {
            a.br.p[r] = static_cast<const T*>(P.br[r]);
            a.r.p[r] = rr[r];
            a.xr.p[r] = xr[r];
        }
        hipLaunchKernelGGL(init_kernel<T>, dim3(nb, ns), dim3(kThr), 0, s, n, a, P);
    }
    hipError_t e = vcycle(vb, za, rr, zr);
    if (e != hipSuccess) return e;
    if ((e = dots(vb, za)) != hipSuccess) return e;
    hipLaunchKernelGGL(coef_kernel, dim3(1), dim3(64), 0, s, st, sumsA, sumsB, nc, nr, 1);
    if (nr)
        hipLaunchKernelGGL(cg_update2_kernel<T>, dim3(nb, nr), dim3(kThr), 0, s, n, cv(zr, nr), mv(pr, nr), st, nc, 1);

    T** z = za;
    T** zn = zb;
    T** v = vb;
    T** vp = vpb;
    T** w = wb;
    T** wp = wpb;
    for (int it = 0; it < iters; ++it) {
        // vector variants (16-byte loads) when rows split into whole vectors
        constexpr int VX = sizeof(T) == 4 ? 4 : 2;
        const bool vec = L0.nx % VX == 0;
        if (nc) {
            if (vec)
                hipLaunchKernelGGL((saddle_apply_v_kernel<T, VX>), dim3(nb, nc), dim3(kThr), 0, s, L0, n, cv(z, nc),
                                   mv(szb, nc), st, P, partA, ns);
            else
                hipLaunchKernelGGL(saddle_apply_kernel<T>, dim3(nb, nc), dim3(kThr), 0, s, L0, n, cv(z, nc),
                                   mv(szb, nc), st, P, partA, ns);
        }
        if (nr) {
            if (vec)
                hipLaunchKernelGGL((cg_apply_v_kernel<T, VX>), dim3(nb, nr), dim3(kThr), 0, s, L0, n, cv(pr, nr),
                                   mv(qr, nr), P, partA, ns);
            else
                hipLaunchKernelGGL(cg_apply_kernel<T>, dim3(nb, nr), dim3(kThr), 0, s, L0, n, cv(pr, nr), mv(qr, nr),
                                   P, partA, ns);
        }
        if ((e = launch_reduce(partA, nb, ns, ns, sumsA, s)) != hipSuccess) return e;
        if (nc)
            hipLaunchKernelGGL(lanczos_kernel<T>, dim3(nb, nc), dim3(kThr), 0, s, 2 * n, cv(szb, nc), cv(v, nc),
                               mv(vp, nc), st, sumsA);
        if (nr)
            hipLaunchKernelGGL(cg_update1_kernel<T>, dim3(nb, nr), dim3(kThr), 0, s, n, cv(pr, nr), cv(qr, nr),
                               mv(xr, nr), mv(rr, nr), st, sumsA, nc);
        // vp now holds v_{j+1}
        if ((e = vcycle(vp, zn, rr, zr)) != hipSuccess) return e;
        if ((e = dots(vp, zn)) != hipSuccess) return e;
        hipLaunchKernelGGL(coef_kernel, dim3(1), dim3(64), 0, s, st, sumsA, sumsB, nc, nr, 0);
        if (nc)
            hipLaunchKernelGGL(minres_update_kernel<T>, dim3(nb, nc), dim3(kThr), 0, s, 2 * n, cv(z, nc), cv(w, nc),
                               mv(wp, nc), mv(xcb, nc), st);
        if (nr)
            hipLaunchKernelGGL(cg_update2_kernel<T>, dim3(nb, nr), dim3(kThr), 0, s, n, cv(zr, nr), mv(pr, nr), st, nc,
                               0);
        std::swap(v, vp);  // v_prev <- v, v <- v_{j+1}
        std::swap(w, wp);  // w_prev <- w, w <- w_{j+1}
        std::swap(z, zn);
    }
    hipLaunchKernelGGL(final_kernel<T>, dim3(nb, ns), dim3(kThr), 0, s, n, cv(xcb, nc), cv(xr, nr), P);
    return hipGetLastError();
}

}  // namespace

size_t sp_ws_bytes(const MgHierarchy& h, long long n, int nc, int nr, bool f32) {
    return f32 ? ws_bytes_t<float>(h, n, nc, nr) : ws_bytes_t<double>(h, n, nc, nr);
}

hipError_t sp_solve(const SpProblem& P, int iters, bool f32, void* ws, hipStream_t s) {
    char* w = static_cast<char*>(ws);
    return f32 ? solve_t<float>(P, iters, w, s) : solve_t<double>(P, iters, w, s);
}

}  // namespace ac
