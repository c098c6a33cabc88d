// Dense products of the exact constant-coefficient solve (Appendix A): the half sine
// matrices applied to every plane column, C = op(S) B with S square (d x d,
// column-major, leading dimension d), B and C d x N column blocks of leading
// dimension ldb / ldc; op(S) = S for the forward transform and S^T for the inverse.
//
// Matrix cores: v_mfma_f64_16x16x4f64 (float64) or v_mfma_f32_16x16x4f32 (float32).
// A workgroup of four waves owns a 128 x 128 tile of C, each wave a 64 x 64 quarter
// held as 4 x 4 accumulator tiles of 16 x 16.  K advances in chunks of 32: a chunk
// of op(S) (32 x 128) and of B (32 x 128) is fetched from global memory into
// registers while the previous chunk, staged in LDS, feeds the matrix cores.
//
// Fragment layouts of the 16x16x4 instructions (one element per lane for A and B,
// four per lane for the 16 x 16 result): lane l = c + 16 g holds A[c][g] and B[g][c];
// result register r of lane l holds C[g + 4 r][c] (float64) or C[4 g + r][c] (float32),
// as measured on gfx950.
//
// LDS: op(S) chunk k-major with a row pitch of 144 elements (the four k rows read
// by one fragment fall on distinct banks), or for S^T row-major with a pitch of 34 as
// B; B chunk column-major with a pitch of 34 (16-byte aligned columns; the sixteen
// columns read by one fragment on distinct banks).
//
// Tile order is XCD-aware: the tiles are cut into eight contiguous ranges, one per XCD
// (workgroups are dealt round-robin to the XCDs), with the row tiles of one column
// block adjacent, so each column block of B is read into one XCD's L2 and reused there.
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

constexpr int kBM = 128, kBN = 128, kBK = 32;
constexpr int kPA = kBM + 16;  // LDS pitch of the op(S) chunk (per k row)
constexpr int kPB = kBK + 2;   // LDS pitch of the B chunk (per column)

typedef double D4 __attribute__((ext_vector_type(4)));
typedef float F4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef D4 Acc;
    static __device__ __forceinline__ Acc run(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef F4 Acc;
    static __device__ __forceinline__ Acc run(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

// Per-thread share of one chunk, in 16-byte pieces of W = 16 / sizeof(T) elements:
//  op(S) = S: row k of the chunk is kBM contiguous elements of column k of S; each
//    pass of the workgroup covers 256 / (kBM / W) rows with consecutive threads on
//    consecutive pieces (16 per thread in all);
//  op(S) = S^T: output row i of the chunk is kBK contiguous elements of column i of
//    S, laid out like B;
//  B: column j of the chunk is kBK contiguous elements; each pass covers
//    256 / (kBK / W) columns, consecutive threads on consecutive pieces (BN / 8
//    elements per thread).
// Consecutive threads thus read and stage consecutive 16-byte pieces (coalesced loads,
// LDS writes without bank conflicts).  FAST: the chunk lies inside both operands and
// every piece starts on a 16-byte boundary, so pieces are fetched as vectors without
// checks; otherwise element by element with zero fill.
template <typename T>
struct Piece {
    static constexpr int W = 16 / sizeof(T);
    typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
};

template <typename T>
__device__ __forceinline__ void load_piece(const T* src, int valid, bool fast, T* dst) {
    constexpr int W = Piece<T>::W;
    if (fast) {
        const typename Piece<T>::V v = *reinterpret_cast<const typename Piece<T>::V*>(src);
#pragma unroll
        for (int u = 0; u < W; ++u) dst[u] = v[u];
    } else {
#pragma unroll
        for (int u = 0; u < W; ++u) dst[u] = u < valid ? src[u] : T(0);
    }
}

template <typename T, bool TRANS, int BN, bool FAST>
__device__ __forceinline__ void fetch_chunk(const T* __restrict__ S, int d, const T* __restrict__ B, int ldb, int N,
                                            int i0, int j0, int k0, T (&ra)[16], T (&rb)[BN / 8]) {
    constexpr int W = Piece<T>::W;
    const int t = threadIdx.x;
    constexpr bool fast = FAST;
    if (!TRANS) {
        constexpr int PR = kBM / W, RP = 256 / PR;  // pieces per row, rows per pass
#pragma unroll
        for (int q = 0; q < 16 / W; ++q) {
            const int k = k0 + q * RP + t / PR, i = i0 + (t % PR) * W;
            load_piece<T>(S + static_cast<long long>(k) * d + i, k < d ? d - i : 0, fast, ra + q * W);
        }
    } else {
        constexpr int PR = kBK / W, RP = 256 / PR;  // pieces per output row, rows per pass
#pragma unroll
        for (int q = 0; q < 16 / W; ++q) {
            const int i = i0 + q * RP + t / PR, k = k0 + (t % PR) * W;
            load_piece<T>(S + static_cast<long long>(i) * d + k, i < d ? d - k : 0, fast, ra + q * W);
        }
    }
    constexpr int PC = kBK / W, CP = 256 / PC;  // pieces per column, columns per pass
#pragma unroll
    for (int q = 0; q < BN / 8 / W; ++q) {
        const int j = j0 + q * CP + t / PC, k = k0 + (t % PC) * W;
        load_piece<T>(B + static_cast<long long>(j) * ldb + k, j < N ? d - k : 0, fast, rb + q * W);
    }
}

template <typename T, bool TRANS, int BN>
__device__ __forceinline__ void stage_chunk(T* As, T* Bs, const T (&ra)[16], const T (&rb)[BN / 8]) {
    constexpr int W = Piece<T>::W;
    const int t = threadIdx.x;
    if (!TRANS) {
        constexpr int PR = kBM / W, RP = 256 / PR;
#pragma unroll
        for (int q = 0; q < 16 / W; ++q) {
            T* dst = As + (q * RP + t / PR) * kPA + (t % PR) * W;
#pragma unroll
            for (int u = 0; u < W; ++u) dst[u] = ra[q * W + u];
        }
    } else {
        constexpr int PR = kBK / W, RP = 256 / PR;
#pragma unroll
        for (int q = 0; q < 16 / W; ++q) {
            T* dst = As + (q * RP + t / PR) * kPB + (t % PR) * W;
#pragma unroll
            for (int u = 0; u < W; ++u) dst[u] = ra[q * W + u];
        }
    }
    constexpr int PC = kBK / W, CP = 256 / PC;
#pragma unroll
    for (int q = 0; q < BN / 8 / W; ++q) {
        T* dst = Bs + (q * CP + t / PC) * kPB + (t % PC) * W;
#pragma unroll
        for (int u = 0; u < W; ++u) dst[u] = rb[q * W + u];
    }
}

// One 128 x BN tile of C.  FAST: the whole tile and every chunk lie inside the
// operands and the pieces are 16-byte aligned (no checks in the loop).
template <typename T, bool TRANS, int BN, bool FAST>
__device__ __forceinline__ void sine_gemm_tile(const T* __restrict__ S, int d, const T* __restrict__ B, int ldb,
                                               T* __restrict__ C, int ldc, int N, int i0, int j0, T* As, T* Bs) {
    using Acc = typename Mfma<T>::Acc;
    constexpr int NT = BN / 32;  // 16-column tiles per wave
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = (w >> 1) * 64, wn = (w & 1) * (BN / 2);
    const int c = lane & 15, g = lane >> 4;

    Acc acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = Acc{0, 0, 0, 0};

    T ra[16], rb[BN / 8];
    fetch_chunk<T, TRANS, BN, FAST>(S, d, B, ldb, N, i0, j0, 0, ra, rb);
    stage_chunk<T, TRANS, BN>(As, Bs, ra, rb);
    __syncthreads();
    const int nchunk = (d + kBK - 1) / kBK;
    for (int ch = 0; ch < nchunk; ++ch) {
        const bool more = ch + 1 < nchunk;
        if (more) fetch_chunk<T, TRANS, BN, FAST>(S, d, B, ldb, N, i0, j0, (ch + 1) * kBK, ra, rb);
#pragma unroll
        for (int ks = 0; ks < kBK / 4; ++ks) {
            const int kr = ks * 4 + g;
            T fa[4], fb[NT];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                fa[mt] = TRANS ? As[(wm + mt * 16 + c) * kPB + kr] : As[kr * kPA + wm + mt * 16 + c];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) fb[nt] = Bs[(wn + nt * 16 + c) * kPB + kr];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = Mfma<T>::run(fa[mt], fb[nt], acc[mt][nt]);
        }
        __syncthreads();
        if (more) {
            stage_chunk<T, TRANS, BN>(As, Bs, ra, rb);
            __syncthreads();
        }
    }
    // lane (c, g) holds four rows of column c of every 16 x 16 tile
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int j = j0 + wn + nt * 16 + c;
        if (!FAST && j >= N) continue;
        T* col = C + static_cast<long long>(j) * ldc;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int i = i0 + wm + mt * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ir = i + Mfma<T>::row(g, r);
                if (FAST || ir < d) col[ir] = acc[mt][nt][r];
            }
        }
    }
}

// BN: columns of the workgroup tile (128 or 64); each wave owns 64 x BN / 2.
template <typename T, bool TRANS, int BN>
__global__ __launch_bounds__(256, 2) void sine_gemm_kernel(const T* __restrict__ S, int d, const T* __restrict__ B,
                                                            int ldb, T* __restrict__ C, int ldc, int N, int tiles_m,
                                                            int tiles, int per_xcd, int aligned) {
    __shared__ T As[kBK * kPA];
    __shared__ T Bs[BN * kPB];
    const int b = blockIdx.x;
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile >= tiles) return;
    const int i0 = (tile % tiles_m) * kBM, j0 = (tile / tiles_m) * BN;
    if (aligned && i0 + kBM <= d && d % kBK == 0 && j0 + BN <= N)
        sine_gemm_tile<T, TRANS, BN, true>(S, d, B, ldb, C, ldc, N, i0, j0, As, Bs);
    else
        sine_gemm_tile<T, TRANS, BN, false>(S, d, B, ldb, C, ldc, N, i0, j0, As, Bs);
}

template <typename T, int BN>
hipError_t sine_gemm_bn(bool trans, const T* S, int d, const T* B, int ldb, T* C, int ldc, int N, hipStream_t s) {
    const int tiles_m = (d + kBM - 1) / kBM;
    const long long tl = static_cast<long long>(tiles_m) * ((N + BN - 1) / BN);
    if (tl > (1LL << 30)) return hipErrorInvalidValue;
    const int tiles = static_cast<int>(tl);
    const int per_xcd = (tiles + 7) / 8;
    const dim3 grid(8 * per_xcd), block(256);
    constexpr size_t A16 = 16 / sizeof(T);
    const int aligned = (reinterpret_cast<size_t>(S) % 16 == 0 && reinterpret_cast<size_t>(B) % 16 == 0 &&
                         d % A16 == 0 && ldb % A16 == 0) ? 1 : 0;
    if (trans) hipLaunchKernelGGL((sine_gemm_kernel<T, true, BN>), grid, block, 0, s, S, d, B, ldb, C, ldc, N, tiles_m, tiles, per_xcd, aligned);
    else hipLaunchKernelGGL((sine_gemm_kernel<T, false, BN>), grid, block, 0, s, S, d, B, ldb, C, ldc, N, tiles_m, tiles, per_xcd, aligned);
    return hipGetLastError();
}

// Tile width: float64 always 64 columns (the 128-column tile would not fit its
// registers with the staging of a chunk); float32 the wider tile unless the narrower
// one leaves less of the last round idle, counting the workgroups the GPU holds at
// once (256 CUs, four per CU).
template <typename T>
hipError_t sine_gemm_t(bool trans, const void* S, int d, const void* B, int ldb, void* C, int ldc, int N,
                       hipStream_t s) {
    constexpr long long kSlots = 1024;
    const long long tm = (d + kBM - 1) / kBM;
    auto idle = [&](int bn) {
        const long long t = tm * ((N + bn - 1) / bn);
        return static_cast<double>((t + kSlots - 1) / kSlots * kSlots - t) / static_cast<double>((t + kSlots - 1) / kSlots * kSlots);
    };
    const T* s_ = static_cast<const T*>(S);
    const T* b_ = static_cast<const T*>(B);
    T* c_ = static_cast<T*>(C);
    if constexpr (sizeof(T) == 8) {
        return sine_gemm_bn<T, 64>(trans, s_, d, b_, ldb, c_, ldc, N, s);
    } else {
        if (idle(64) + 0.05 < idle(128)) return sine_gemm_bn<T, 64>(trans, s_, d, b_, ldb, c_, ldc, N, s);
        return sine_gemm_bn<T, 128>(trans, s_, d, b_, ldb, c_, ldc, N, s);
    }
}

}  // namespace

hipError_t launch_sine_gemm(int prec, bool trans, const void* S, int d, const void* B, int ldb, void* C, int ldc,
                            int N, hipStream_t s) {
    if (d < 1 || N < 1 || ldb < d || ldc < d) return hipErrorInvalidValue;
    return prec == 0 ? sine_gemm_t<double>(trans, S, d, B, ldb, C, ldc, N, s)
                     : sine_gemm_t<float>(trans, S, d, B, ldb, C, ldc, N, s);
}

}  // namespace ac
