// Learned warm start for the shifted inner solves: a three-layer 3x3 convolutional
// network (5 -> 16 -> 16 -> 2 channels, ReLU after the first two layers), bfloat16
// weights and activations, float32 accumulation on the matrix cores.
//
// Activations are NHWC with 16 channels per pixel (bf16 bits in uint16_t).  A 3x3
// convolution is nine chained 16x16x16 MFMAs per 16-pixel tile: for tap t the A
// operand holds 16 pixels x 16 input channels shifted by the tap offset, the B
// operand the 16x16 weight matrix of that tap.  The input gradient is the same
// convolution with flipped, transposed weights; the weight gradient reduces over
// pixels on the matrix cores after an LDS transpose of each 16-pixel block.
//
// Operand layouts of v_mfma_f32_16x16x16_bf16 (wave64): lane l holds
//   A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16], D[4 (l / 16) + j][l % 16], j = 0..3.
#include <hip/hip_runtime.h>

#include "ac_internal.h"

namespace ac {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 16;  // channels per pixel in every activation tensor

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

__device__ __forceinline__ bf16x4 ld4(const uint16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }

// 16 bf16 values -> two 16-byte stores
__device__ __forceinline__ void store16(uint16_t* dst, const uint16_t (&h)[kC]) {
    uint4 a, b;
    a.x = h[0] | (static_cast<uint32_t>(h[1]) << 16);
    a.y = h[2] | (static_cast<uint32_t>(h[3]) << 16);
    a.z = h[4] | (static_cast<uint32_t>(h[5]) << 16);
    a.w = h[6] | (static_cast<uint32_t>(h[7]) << 16);
    b.x = h[8] | (static_cast<uint32_t>(h[9]) << 16);
    b.y = h[10] | (static_cast<uint32_t>(h[11]) << 16);
    b.z = h[12] | (static_cast<uint32_t>(h[13]) << 16);
    b.w = h[14] | (static_cast<uint32_t>(h[15]) << 16);
    reinterpret_cast<uint4*>(dst)[0] = a;
    reinterpret_cast<uint4*>(dst)[1] = b;
}

// ---------------------------------------------------------------------------
// 3x3 convolution, one wave per tile of 16 consecutive pixels of one row.
__global__ __launch_bounds__(256) void conv3x3_kernel(const CnnConvArgs a) {
    const long long ntx = (a.W + 15) / 16;
    const long long ntiles = static_cast<long long>(a.B) * a.H * ntx;
    const long long tile = static_cast<long long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    const int xt = static_cast<int>(tile % ntx);
    const long long rest = tile / ntx;
    const int y = static_cast<int>(rest % a.H);
    const int b = static_cast<int>(rest / a.H);
    const int x0 = xt * 16;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y + t / 3 - 1;
        const int xx = x0 + i + t % 3 - 1;
        bf16x4 av = {0, 0, 0, 0};
        if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
            av = ld4(a.in + ((static_cast<long long>(b) * a.H + yy) * a.W + xx) * kC + 4 * g);
        const bf16x4 bv = ld4(a.w + (t * kC + i) * kC + 4 * g);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    // lane holds output channel i of pixels x0 + 4g + j
    const float bias = a.bias ? a.bias[i] : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int px = x0 + 4 * g + j;
        if (px >= a.W) continue;
        const long long pix = (static_cast<long long>(b) * a.H + y) * a.W + px;
        float v = acc[j] + bias;
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.mask && !(bf2f(a.mask[pix * kC + i]) > 0.f)) v = 0.f;
        if (a.out16) a.out16[pix * kC + i] = f2bf(v);
        if (a.out32 && i < a.nout) a.out32[pix * a.nout + i] = v;
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients: dW[t][o][c] = sum_p act[p + off_t][c] dz[p][o],
// db[o] = sum_p dz[p][o].  Each wave accumulates the nine 16x16 tap blocks over its
// share of tiles and writes a partial; a second kernel reduces the partials in a
// fixed order.  All waves of a block run the same trip count (barriers).
__global__ __launch_bounds__(256) void wgrad_kernel(const CnnWgradArgs a) {
    __shared__ uint16_t dzs[4][16 * kC];
    __shared__ uint16_t acts[4][3 * 18 * kC];
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    const long long ntx = (a.W + 15) / 16;
    const long long ntiles = static_cast<long long>(a.B) * a.H * ntx;
    const long long nwaves = static_cast<long long>(gridDim.x) * 4;
    const long long gw = static_cast<long long>(blockIdx.x) * 4 + wv;
    const long long trips = (ntiles + nwaves - 1) / nwaves;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = {0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    for (long long it = 0; it < trips; ++it) {
        const long long tile = gw + it * nwaves;
        const bool ok = tile < ntiles;
        int x0 = 0, y = 0, b = 0;
        if (ok) {
            x0 = static_cast<int>(tile % ntx) * 16;
            const long long rest = tile / ntx;
            y = static_cast<int>(rest % a.H);
            b = static_cast<int>(rest / a.H);
        }
        // dz block: 16 pixels x 16 channels
        {
            bf16x4 v = {0, 0, 0, 0};
            const int px = x0 + i;
            if (ok && px < a.W) v = ld4(a.dz + ((static_cast<long long>(b) * a.H + y) * a.W + px) * kC + 4 * g);
            *reinterpret_cast<bf16x4*>(&dzs[wv][i * kC + 4 * g]) = v;
        }
        // activation halo region: rows y-1..y+1, pixels x0-1..x0+16
        for (int c = lane; c < 3 * 18 * 4; c += 64) {
            const int r = c / 72, rem = c % 72, px = rem / 4, g4 = rem % 4;
            const int yy = y + r - 1, xx = x0 + px - 1;
            bf16x4 v = {0, 0, 0, 0};
            if (ok && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                v = ld4(a.act + ((static_cast<long long>(b) * a.H + yy) * a.W + xx) * kC + 4 * g4);
            *reinterpret_cast<bf16x4*>(&acts[wv][(r * 18 + px) * kC + 4 * g4]) = v;
        }
        __syncthreads();
        // A = dz^T (M = output channel i, K = pixel), bias partial from the same values
        bf16x4 av;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint16_t u = dzs[wv][(4 * g + j) * kC + i];
            av[j] = static_cast<short>(u);
            bacc += bf2f(u);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            bf16x4 bv;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bv[j] = static_cast<short>(acts[wv][((1 + dy) * 18 + (4 * g + j) + 1 + dx) * kC + i]);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
    // D[o = 4g + j][c = i] of tap t
    float* out = a.partial + gw * (9 * 256 + 16);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[t * 256 + (4 * g + j) * kC + i] = acc[t][j];
    // bias: lanes i, i+16, i+32, i+48 hold disjoint pixel subsets of channel i
    bacc += __shfl_down(bacc, 32, 64);
    bacc += __shfl_down(bacc, 16, 64);
    if (lane < 16) out[9 * 256 + lane] = bacc;
}

__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* __restrict__ partial, long long nwaves,
                                                           float* __restrict__ grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 9 * 256 + 16) return;
    double s = 0.0;
    for (long long w = 0; w < nwaves; ++w) s += partial[w * (9 * 256 + 16) + q];
    grad[q] = static_cast<float>(s);
}

// ---------------------------------------------------------------------------
// Masked relative squared error and its gradient (channels 0, 1; others zero).
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                   const float* __restrict__ tnorm, int B, int H, int W, int border,
                                                   uint16_t* __restrict__ dy16, float* __restrict__ partial) {
    const long long npix = static_cast<long long>(B) * H * W;
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (p < npix) {
        const int x = static_cast<int>(p % W);
        const int yy = static_cast<int>((p / W) % H);
        const int b = static_cast<int>(p / (static_cast<long long>(W) * H));
        const bool in = x >= border && x < W - border && yy >= border && yy < H - border;
        const float inv = 1.f / tnorm[b];
        uint16_t g[kC];
#pragma unroll
        for (int c = 0; c < kC; ++c) g[c] = 0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float d = in ? (y[p * 2 + c] - t[p * 2 + c]) : 0.f;
            l += d * d * inv;
            g[c] = f2bf(2.f * d * inv / static_cast<float>(B));
        }
        store16(dy16 + p * kC, g);
    }
    // block sum
    __shared__ float red[4];
    for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// Residual-space loss on crops: e = M (rhat - (A - lambda) y), A the five-point
// operator of the crop's coefficients with face values (kappa_i + kappa_nb)/2.  With
// border >= 1 every masked point has its four neighbours inside the crop.  Writes e
// (zero outside the mask) and per-block sums of |e|^2 / rnorm_b.
__global__ __launch_bounds__(256) void resloss_kernel(const float2* __restrict__ y, const float2* __restrict__ rhat,
                                                      const float* __restrict__ kap, const float2* __restrict__ lam,
                                                      const float* __restrict__ rnorm, int B, int H, int W,
                                                      int border, float2* __restrict__ e,
                                                      float* __restrict__ partial) {
    const long long npix = static_cast<long long>(B) * H * W;
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (p < npix) {
        const int x = static_cast<int>(p % W);
        const int yy = static_cast<int>((p / W) % H);
        const int b = static_cast<int>(p / (static_cast<long long>(W) * H));
        float2 ev = make_float2(0.f, 0.f);
        if (x >= border && x < W - border && yy >= border && yy < H - border) {
            const float k0 = kap[p];
            const float2 yc = y[p];
            const long long nb[4] = {p - 1, p + 1, p - W, p + W};
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const float kf = 0.5f * (k0 + kap[nb[f]]);
                const float2 yn = y[nb[f]];
                ar += kf * (yc.x - yn.x);
                ai += kf * (yc.y - yn.y);
            }
            const float2 lm = lam[b];
            const float br = yc.x + ar - (lm.x * yc.x - lm.y * yc.y);
            const float bi = yc.y + ai - (lm.x * yc.y + lm.y * yc.x);
            const float2 r = rhat[p];
            ev = make_float2(r.x - br, r.y - bi);
            l = (ev.x * ev.x + ev.y * ev.y) / rnorm[b];
        }
        e[p] = ev;
    }
    __shared__ float red[4];
    for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// dL/dy = -2 (A - conj(lambda)) e / (B rnorm_b) (A is symmetric), as bf16 into
// channels 0, 1 of the 16-channel gradient tensor.  Faces to points outside the crop
// are skipped: e vanishes there and at every unmasked point, so they add nothing.
__global__ __launch_bounds__(256) void resgrad_kernel(const float2* __restrict__ e, const float* __restrict__ kap,
                                                      const float2* __restrict__ lam, const float* __restrict__ rnorm,
                                                      int B, int H, int W, uint16_t* __restrict__ dy16) {
    const long long npix = static_cast<long long>(B) * H * W;
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int x = static_cast<int>(p % W);
    const int yy = static_cast<int>((p / W) % H);
    const int b = static_cast<int>(p / (static_cast<long long>(W) * H));
    const float k0 = kap[p];
    const float2 ec = e[p];
    float ar = 0.f, ai = 0.f;
    const bool ok[4] = {x > 0, x < W - 1, yy > 0, yy < H - 1};
    const long long nb[4] = {p - 1, p + 1, p - W, p + W};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (!ok[f]) continue;
        const float kf = 0.5f * (k0 + kap[nb[f]]);
        const float2 en = e[nb[f]];
        ar += kf * (ec.x - en.x);
        ai += kf * (ec.y - en.y);
    }
    const float2 lm = lam[b];  // conj(lambda) e = (lr e.x + li e.y, lr e.y - li e.x)
    const float gr = ec.x + ar - (lm.x * ec.x + lm.y * ec.y);
    const float gi = ec.y + ai - (lm.x * ec.y - lm.y * ec.x);
    const float sc = -2.f / (static_cast<float>(B) * rnorm[b]);
    uint16_t g[kC];
#pragma unroll
    for (int c = 0; c < kC; ++c) g[c] = 0;
    g[0] = f2bf(sc * gr);
    g[1] = f2bf(sc * gi);
    store16(dy16 + p * kC, g);
}

// ---------------------------------------------------------------------------
// Adam on the float32 master parameters, then the bf16 forward weights
// wf[L][t][n][k] = W_L[t][n][k] and backward weights wb[L][t][c][o] = W_L[8 - t][o][c].
// Parameter vector: [W1 (9x16x16), b1 (16), W2, b2, W3, b3]; entries outside the
// network (input channels >= 5 of layer 1, outputs >= 2 of layer 3) stay zero.
__device__ __forceinline__ bool frozen(int q) {
    const int L = q / 2320, r = q % 2320;
    if (r < 2304) {
        const int o = (r % 256) / 16, c = r % 16;
        if (L == 0 && c >= 5) return true;
        if (L == 2 && o >= 2) return true;
    } else if (L == 2 && r - 2304 >= 2) {
        return true;
    }
    return false;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float bc1, float bc2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kCnnParams) return;
    if (frozen(q)) {
        w[q] = 0.f;
        return;
    }
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
}

__global__ __launch_bounds__(256) void weights_bf16_kernel(const float* __restrict__ w, uint16_t* __restrict__ wf,
                                                           uint16_t* __restrict__ wb, float* __restrict__ bias) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;  // over 3 x 2304
    if (q < 3 * 16) bias[q] = w[(q / 16) * 2320 + 2304 + q % 16];
    if (q >= 3 * 2304) return;
    const int L = q / 2304, r = q % 2304;
    const int t = r / 256, n = (r % 256) / 16, k = r % 16;
    wf[q] = f2bf(w[L * 2320 + r]);
    // wb[L][t][c = n][o = k] = W_L[8 - t][o = k][c = n]
    wb[q] = f2bf(w[L * 2320 + (8 - t) * 256 + k * 16 + n]);
}

// ---------------------------------------------------------------------------
// Inference plumbing.

// Network inputs for every shift slot: X[s][p][0..15] = (Re rhat_s / sc_s, Im rhat_s / sc_s,
// Re lambda_s, Im lambda_s, (ln kappa - c0) / c1, 0, ...).
template <typename R>
__global__ __launch_bounds__(256) void prep_kernel(const CnnPrepArgs a) {
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const float lk = static_cast<float>((log(a.kappa[p]) - a.c0) / a.c1);
    for (int s = 0; s < a.ns; ++s) {
        const R* src = static_cast<const R*>(a.rhat) + a.soff[s];
        float re, im;
        if (a.is_real[s]) {
            re = static_cast<float>(src[p]);
            im = 0.f;
        } else {
            re = static_cast<float>(src[2 * p]);
            im = static_cast<float>(src[2 * p + 1]);
        }
        uint16_t h[kC];
#pragma unroll
        for (int c = 0; c < kC; ++c) h[c] = 0;
        h[0] = f2bf(re * a.inv_scale[s]);
        h[1] = f2bf(im * a.inv_scale[s]);
        h[2] = f2bf(a.lam_re[s]);
        h[3] = f2bf(a.lam_im[s]);
        h[4] = f2bf(lk);
        store16(a.x + (static_cast<long long>(s) * a.n + p) * kC, h);
        if (a.rs) {
            float2 t;
            t.x = re * a.inv_scale[s];
            t.y = im * a.inv_scale[s];
            reinterpret_cast<float2*>(a.rs)[static_cast<long long>(s) * a.n + p] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused inference: the three layers for one 16 x 16 output tile of every shift slot,
// intermediate activations in LDS.  The layer-1 input region is the tile plus a
// 3-pixel ring (22 x 22), built directly from rhat and kappa; layer 1 is evaluated on
// 20 x 20, layer 2 on 18 x 18, layer 3 on the tile.  Region pixels outside the grid
// are zero at every layer (the zero padding of the layer-by-layer evaluation), taps
// are chained in the same order, so the result equals that evaluation.  Each region
// is covered by 16-pixel chunks (flattened row-major), one 9-MFMA chain per chunk.
constexpr int kFT = 16;         // output tile edge
constexpr int kR0 = kFT + 6;    // layer-1 input region edge
constexpr int kR1 = kFT + 4;    // layer-1 output region edge
constexpr int kR2 = kFT + 2;    // layer-2 output region edge

// One layer on the RO x RO output region from the (RO + 2) x (RO + 2) input region;
// (gx0, gy0): grid coordinates of the output region's origin.
template <int RO>
__device__ __forceinline__ void fused_layer(const uint16_t* __restrict__ in, uint16_t* __restrict__ out,
                                            const bf16x4 (&wt)[9], float bias, int gx0, int gy0, int nx, int ny) {
    constexpr int RI = RO + 2;
    constexpr int NPIX = RO * RO;
    constexpr int NCH = (NPIX + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    for (int c = wv; c < NCH; c += 4) {
        const int q = 16 * c + i;  // this lane's A row: output pixel q of the chunk
        const bool qok = q < NPIX;
        const int qy = qok ? q / RO : 0, qx = qok ? q % RO : 0;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            bf16x4 av = {0, 0, 0, 0};
            if (qok) av = *reinterpret_cast<const bf16x4*>(in + ((qy + t / 3) * RI + qx + t % 3) * kC + 4 * g);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, wt[t], acc, 0, 0, 0);
        }
        // lane holds output channel i of chunk pixels 4g + j
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int qq = 16 * c + 4 * g + j;
            if (qq >= NPIX) continue;
            const int oy = qq / RO, ox = qq % RO;
            const int gy = gy0 + oy, gx = gx0 + ox;
            float v = fmaxf(acc[j] + bias, 0.f);
            if (gy < 0 || gy >= ny || gx < 0 || gx >= nx) v = 0.f;
            out[qq * kC + i] = f2bf(v);
        }
    }
}

template <typename R>
__global__ __launch_bounds__(256) void cnn_fused_kernel(const CnnPrepArgs a, const uint16_t* __restrict__ wf,
                                                        const float* __restrict__ bias, void* x0buf) {
    __shared__ __align__(16) uint16_t in0[kR0 * kR0 * kC];
    __shared__ __align__(16) uint16_t in1[kR1 * kR1 * kC];
    __shared__ __align__(16) uint16_t in2[kR2 * kR2 * kC];
    __shared__ uint16_t lks[kR0 * kR0];
    const int nx = a.g.nx, ny = a.g.ny;
    const int ntx = (nx + kFT - 1) / kFT;
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int X0 = tx * kFT - 3, Y0 = ty * kFT - 3;  // grid coordinates of the input region's origin
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    bf16x4 w1[9], w2[9], w3[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        w1[t] = ld4(wf + (t * kC + i) * kC + 4 * g);
        w2[t] = ld4(wf + 2304 + (t * kC + i) * kC + 4 * g);
        w3[t] = ld4(wf + 2 * 2304 + (t * kC + i) * kC + 4 * g);
    }
    const float b1 = bias[i], b2 = bias[16 + i], b3 = bias[32 + i];
    for (int q = threadIdx.x; q < kR0 * kR0; q += blockDim.x) {
        const int gy = Y0 + q / kR0, gx = X0 + q % kR0;
        uint16_t v = 0;
        if (gy >= 0 && gy < ny && gx >= 0 && gx < nx)
            v = f2bf(static_cast<float>((log(a.kappa[static_cast<long long>(gy) * nx + gx]) - a.c0) / a.c1));
        lks[q] = v;
    }
    for (int s = 0; s < a.ns; ++s) {
        __syncthreads();  // lks written; the previous slot's layer-1 reads of in0 are done
        const R* src = static_cast<const R*>(a.rhat) + a.soff[s];
        const bool re_only = a.is_real[s];
        for (int q = threadIdx.x; q < kR0 * kR0; q += blockDim.x) {
            const int gy = Y0 + q / kR0, gx = X0 + q % kR0;
            uint16_t h[kC];
#pragma unroll
            for (int c = 0; c < kC; ++c) h[c] = 0;
            if (gy >= 0 && gy < ny && gx >= 0 && gx < nx) {
                const long long p = static_cast<long long>(gy) * nx + gx;
                const float re = static_cast<float>(re_only ? src[p] : src[2 * p]);
                const float im = re_only ? 0.f : static_cast<float>(src[2 * p + 1]);
                h[0] = f2bf(re * a.inv_scale[s]);
                h[1] = f2bf(im * a.inv_scale[s]);
                h[2] = f2bf(a.lam_re[s]);
                h[3] = f2bf(a.lam_im[s]);
                h[4] = lks[q];
            }
            store16(in0 + q * kC, h);
        }
        __syncthreads();
        fused_layer<kR1>(in0, in1, w1, b1, X0 + 1, Y0 + 1, nx, ny);
        __syncthreads();
        fused_layer<kR2>(in1, in2, w2, b2, X0 + 2, Y0 + 2, nx, ny);
        __syncthreads();
        // layer 3 on the tile: chunk c is tile row c; lanes i = 0, 1 hold Re, Im
        R* dst = static_cast<R*>(x0buf) + a.soff[s];
        const float sc = a.scale[s];
        for (int c = wv; c < kFT; c += 4) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const bf16x4 av = *reinterpret_cast<const bf16x4*>(in2 + ((c + t / 3) * kR2 + i + t % 3) * kC + 4 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, w3[t], acc, 0, 0, 0);
            }
            const int gy = ty * kFT + c;
            if (i < 2 && gy < ny && !(re_only && i == 1)) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int gx = tx * kFT + 4 * g + j;
                    if (gx >= nx) continue;
                    const long long p = static_cast<long long>(gy) * nx + gx;
                    const float v = sc * (acc[j] + b3);
                    if (re_only) dst[p] = static_cast<R>(v);
                    else dst[2 * p + i] = static_cast<R>(v);
                }
            }
        }
    }
}

// x0 slot s = scale_s * (y0 + i y1)
template <typename R>
__global__ __launch_bounds__(256) void post_kernel(const CnnPrepArgs a, const float* __restrict__ y, void* x0buf) {
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    for (int s = 0; s < a.ns; ++s) {
        R* dst = static_cast<R*>(x0buf) + a.soff[s];
        const float* ys = y + (static_cast<long long>(s) * a.n + p) * 2;
        // x0 = scale * c * y with the per-slot complex factor c
        const float cr = a.scale[s] * a.fac_re[s], ci = a.scale[s] * a.fac_im[s];
        if (a.is_real[s]) {
            dst[p] = static_cast<R>(cr * ys[0]);
        } else {
            dst[2 * p] = static_cast<R>(cr * ys[0] - ci * ys[1]);
            dst[2 * p + 1] = static_cast<R>(cr * ys[1] + ci * ys[0]);
        }
    }
}

// Per-slot partial sums, four per slot: |rhat|^2, and with a guess x0 (else zero)
// |B x0|^2, Re and Im of sum conj(B x0) rhat, where B = A - lambda I.  The residual
// of c x0 for any complex c follows: |rhat - c B x0|^2 = |rhat|^2 - 2 Re(c conj-dot)
// + |c|^2 |B x0|^2.  One slot per blockIdx.y (its four sums stay in registers); the
// points of a thread, and so every partial, do not depend on the slot count.
template <typename R, typename KS>
__global__ __launch_bounds__(256) void resid_kernel(const CnnPrepArgs a, const void* x0buf, const void* kap,
                                                    double* partial) {
    const Geom g = a.g;
    const int s = blockIdx.y;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    const KS* k = static_cast<const KS*>(kap);
    auto kv = [&](long long i) -> double {
        if constexpr (sizeof(KS) == 2) return static_cast<double>(bf2f(k[i]));
        else return static_cast<double>(k[i]);
    };
    const R* rh = static_cast<const R*>(a.rhat) + a.soff[s];
    const R* x0 = x0buf ? static_cast<const R*>(x0buf) + a.soff[s] : nullptr;
    const bool re = a.is_real[s];
    const double lr = a.lam_re[s], li = a.lam_im[s];
    constexpr int dxs[4] = {1, -1, 0, 0}, dys[4] = {0, 0, 1, -1};
    const int nd = g.dim == 2 ? 4 : 2;
    for (long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; p < a.n; p += step) {
        const double rr = re ? rh[p] : rh[2 * p], ri = re ? 0.0 : rh[2 * p + 1];
        acc[0] += rr * rr + ri * ri;
        if (!x0) continue;
        const int ix = static_cast<int>(p % g.nx), iy = static_cast<int>(p / g.nx);
        const double kc = kv(p);
        long long nb[4];
        double f[4];
        bool ok[4];
        double diag = 1.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            ok[d] = false;
            nb[d] = p;
            f[d] = 0.0;
            if (d >= nd) continue;
            int jx = ix + dxs[d], jy = iy + dys[d];
            const bool inside = jx >= 0 && jx < g.nx && jy >= 0 && jy < g.ny;
            if (inside || g.periodic) {
                jx = (jx + g.nx) % g.nx;
                jy = (jy + g.ny) % g.ny;
                nb[d] = static_cast<long long>(jy) * g.nx + jx;
                f[d] = 0.5 * (kc + kv(nb[d]));
                diag += f[d];
                ok[d] = true;
            } else {
                diag += kc;
            }
        }
        const double xr = re ? x0[p] : x0[2 * p], xi = re ? 0.0 : x0[2 * p + 1];
        double br = (diag - lr) * xr + li * xi, bi = (diag - lr) * xi - li * xr;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (!ok[d]) continue;
            br -= f[d] * (re ? x0[nb[d]] : x0[2 * nb[d]]);
            bi -= re ? 0.0 : f[d] * x0[2 * nb[d] + 1];
        }
        acc[1] += br * br + bi * bi;
        acc[2] += br * rr + bi * ri;
        acc[3] += br * ri - bi * rr;
    }
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wid][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4)
        partial[blockIdx.x * 4 * kMaxShift + 4 * s + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void zero_slot_kernel(void* buf, long long off_bytes, long long nbytes) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nbytes / 4) reinterpret_cast<uint32_t*>(static_cast<char*>(buf) + off_bytes)[i] = 0u;
}

}  // namespace

int cnn_wgrad_waves(long long ntiles) {
    long long w = ntiles < 2048 ? ntiles : 2048;
    w = (w + 3) / 4 * 4;
    return static_cast<int>(w < 4 ? 4 : w);
}

hipError_t launch_cnn_conv(const CnnConvArgs& a, hipStream_t s) {
    const long long ntiles = static_cast<long long>(a.B) * a.H * ((a.W + 15) / 16);
    const int blocks = static_cast<int>((ntiles + 3) / 4);
    hipLaunchKernelGGL(conv3x3_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cnn_wgrad(const CnnWgradArgs& a, float* grad, hipStream_t s) {
    const long long ntiles = static_cast<long long>(a.B) * a.H * ((a.W + 15) / 16);
    const int waves = cnn_wgrad_waves(ntiles);
    hipLaunchKernelGGL(wgrad_kernel, dim3(waves / 4), dim3(256), 0, s, a);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((9 * 256 + 16 + 255) / 256), dim3(256), 0, s, a.partial,
                       static_cast<long long>(waves), grad);
    return hipGetLastError();
}

hipError_t launch_cnn_loss(const float* y, const float* t, const float* tnorm, int B, int H, int W, int border,
                           uint16_t* dy16, float* partial, int* nblocks, hipStream_t s) {
    const long long npix = static_cast<long long>(B) * H * W;
    const int blocks = static_cast<int>((npix + 255) / 256);
    *nblocks = blocks;
    hipLaunchKernelGGL(loss_kernel, dim3(blocks), dim3(256), 0, s, y, t, tnorm, B, H, W, border, dy16, partial);
    return hipGetLastError();
}

hipError_t launch_cnn_resloss(const float* y, const float* rhat, const float* kap, const float* lam,
                              const float* rnorm, int B, int H, int W, int border, float* e, uint16_t* dy16,
                              float* partial, int* nblocks, hipStream_t s) {
    const long long npix = static_cast<long long>(B) * H * W;
    const int blocks = static_cast<int>((npix + 255) / 256);
    *nblocks = blocks;
    const float2* lm = reinterpret_cast<const float2*>(lam);
    float2* e2 = reinterpret_cast<float2*>(e);
    hipLaunchKernelGGL(resloss_kernel, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const float2*>(y),
                       reinterpret_cast<const float2*>(rhat), kap, lm, rnorm, B, H, W, border, e2, partial);
    hipLaunchKernelGGL(resgrad_kernel, dim3(blocks), dim3(256), 0, s, e2, kap, lm, rnorm, B, H, W, dy16);
    return hipGetLastError();
}

hipError_t launch_cnn_adam(float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                           float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, w, g, m, v, lr, b1, b2, eps,
                       bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_cnn_weights(const float* w, uint16_t* wf, uint16_t* wb, float* bias, hipStream_t s) {
    hipLaunchKernelGGL(weights_bf16_kernel, dim3((3 * 2304 + 255) / 256), dim3(256), 0, s, w, wf, wb, bias);
    return hipGetLastError();
}

hipError_t launch_cnn_prep(int prec, const CnnPrepArgs& a, hipStream_t s) {
    const int blocks = static_cast<int>((a.n + 255) / 256);
    if (prec == 0) hipLaunchKernelGGL(prep_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(prep_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cnn_fused(int prec, const CnnPrepArgs& a, const uint16_t* wf, const float* bias, void* x0buf,
                            hipStream_t s) {
    const int tiles = ((a.g.nx + kFT - 1) / kFT) * ((a.g.ny + kFT - 1) / kFT);
    if (prec == 0) hipLaunchKernelGGL(cnn_fused_kernel<double>, dim3(tiles), dim3(256), 0, s, a, wf, bias, x0buf);
    else hipLaunchKernelGGL(cnn_fused_kernel<float>, dim3(tiles), dim3(256), 0, s, a, wf, bias, x0buf);
    return hipGetLastError();
}

hipError_t launch_cnn_post(int prec, const CnnPrepArgs& a, const float* y, void* x0buf, hipStream_t s) {
    const int blocks = static_cast<int>((a.n + 255) / 256);
    if (prec == 0) hipLaunchKernelGGL(post_kernel<double>, dim3(blocks), dim3(256), 0, s, a, y, x0buf);
    else hipLaunchKernelGGL(post_kernel<float>, dim3(blocks), dim3(256), 0, s, a, y, x0buf);
    return hipGetLastError();
}

hipError_t launch_cnn_resid(int prec, const CnnPrepArgs& a, const void* x0buf, const void* kap, double* partial,
                            int nblk, hipStream_t s) {
    if (a.ns < 1 || a.ns > kMaxShift) return hipErrorInvalidValue;
    const dim3 grid(nblk, a.ns);
    if (prec == 0) hipLaunchKernelGGL((resid_kernel<double, double>), grid, dim3(256), 0, s, a, x0buf, kap, partial);
    else if (prec == 1) hipLaunchKernelGGL((resid_kernel<float, uint16_t>), grid, dim3(256), 0, s, a, x0buf, kap, partial);
    else hipLaunchKernelGGL((resid_kernel<float, float>), grid, dim3(256), 0, s, a, x0buf, kap, partial);
    return hipGetLastError();
}

hipError_t launch_zero_bytes(void* buf, long long off_bytes, long long nbytes, hipStream_t s) {
    const long long words = nbytes / 4;
    hipLaunchKernelGGL(zero_slot_kernel, dim3(static_cast<int>((words + 255) / 256)), dim3(256), 0, s, buf, off_bytes,
                       nbytes);
    return hipGetLastError();
}

}  // namespace ac
