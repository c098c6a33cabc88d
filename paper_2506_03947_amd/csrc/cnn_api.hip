// C ABI of alphacirc: the learned warm start (network parameters, training steps,
// inputs and guesses).
#include "host.h"

using namespace ach;

// ---------------------------------------------------------------------------
// warm-start network

namespace {
size_t cnn_train_ws_bytes(long long B, long long H, long long W) {
    const size_t px = static_cast<size_t>(B * H * W);
    const long long tiles = B * H * ((W + 15) / 16);
    return 5 * align_up(px * 32, 256) + align_up(px * 8, 256) +
           align_up(static_cast<size_t>(ac::cnn_wgrad_waves(tiles)) * (9 * 256 + 16) * sizeof(float), 256) +
           align_up(static_cast<size_t>((px + 255) / 256) * sizeof(float), 256) + 256;
}
int cnn_check_shape(int B, int H, int W) {
    if (B < 1 || H < 1 || W < 1) return fail(AC_ERR_ARG, "batch and image sizes must be positive");
    if (static_cast<long long>(B) * H * W > (1LL << 31)) return fail(AC_ERR_UNSUPPORTED, "batch too large");
    return AC_OK;
}
}  // namespace

int ac_cnn_param_count(void) { return ac::kCnnParams; }

int ac_cnn_create(ac_ctx* c, ac_cnn** out) {
    if (!c || !out) return fail(AC_ERR_ARG, "NULL argument");
    *out = nullptr;
    AC_HIP(hipSetDevice(c->device));
    auto* n = new ac_cnn();
    n->ctx = c;
    const size_t P = ac::kCnnParams;
    const size_t bytes = 4 * align_up(P * 4, 256) + 2 * align_up(3 * 2304 * 2, 256) + 256;
    hipError_t e = hipMalloc(&n->mem, bytes);
    if (e != hipSuccess) {
        delete n;
        return fail(AC_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    char* b = n->mem;
    n->w = reinterpret_cast<float*>(b);
    b += align_up(P * 4, 256);
    n->g = reinterpret_cast<float*>(b);
    b += align_up(P * 4, 256);
    n->m = reinterpret_cast<float*>(b);
    b += align_up(P * 4, 256);
    n->v = reinterpret_cast<float*>(b);
    b += align_up(P * 4, 256);
    n->wf = reinterpret_cast<uint16_t*>(b);
    b += align_up(3 * 2304 * 2, 256);
    n->wb = reinterpret_cast<uint16_t*>(b);
    b += align_up(3 * 2304 * 2, 256);
    n->bias = reinterpret_cast<float*>(b);
    e = launch_zero(reinterpret_cast<double*>(n->mem), static_cast<long long>(bytes / 8), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(n->mem);
        delete n;
        return fail(AC_ERR_HIP, std::string("cnn init: ") + hipGetErrorString(e));
    }
    *out = n;
    return AC_OK;
}

int ac_cnn_destroy(ac_cnn* n) {
    if (!n) return AC_OK;
    (void)hipSetDevice(n->ctx->device);
    (void)hipStreamSynchronize(n->ctx->stream);
    (void)hipFree(n->mem);
    delete n;
    return AC_OK;
}

int ac_cnn_set_params(ac_cnn* n, const float* params, double c0, double c1) {
    if (!n || !params) return fail(AC_ERR_ARG, "NULL argument");
    if (!(c1 > 0.0) || !std::isfinite(c0) || !std::isfinite(c1)) return fail(AC_ERR_ARG, "need finite c0 and c1 > 0");
    for (int q = 0; q < ac::kCnnParams; ++q)
        if (!std::isfinite(params[q])) return fail(AC_ERR_NONFINITE, "parameters must be finite");
    AC_HIP(hipSetDevice(n->ctx->device));
    hipStream_t st = n->ctx->stream;
    AC_HIP(hipMemcpyAsync(n->w, params, ac::kCnnParams * sizeof(float), hipMemcpyHostToDevice, st));
    const size_t P = ac::kCnnParams;
    AC_HIP(launch_zero(reinterpret_cast<double*>(n->m), static_cast<long long>(P / 2), st));
    AC_HIP(launch_zero(reinterpret_cast<double*>(n->v), static_cast<long long>(P / 2), st));
    // entries outside the network are forced to zero by an Adam step of size 0
    AC_HIP(ac::launch_cnn_adam(n->w, n->g, n->m, n->v, 0.f, 0.9f, 0.999f, 1e-8f, 1.f, 1.f, st));
    AC_HIP(ac::launch_cnn_weights(n->w, n->wf, n->wb, n->bias, st));
    AC_HIP(hipStreamSynchronize(st));
    n->c0 = c0;
    n->c1 = c1;
    n->t = 0;
    return AC_OK;
}

int ac_cnn_get_params(const ac_cnn* n, float* params, double* c0, double* c1) {
    if (!n) return fail(AC_ERR_ARG, "NULL argument");
    AC_HIP(hipSetDevice(n->ctx->device));
    if (params) {
        AC_HIP(hipMemcpyAsync(params, n->w, ac::kCnnParams * sizeof(float), hipMemcpyDeviceToHost, n->ctx->stream));
        AC_HIP(hipStreamSynchronize(n->ctx->stream));
    }
    if (c0) *c0 = n->c0;
    if (c1) *c1 = n->c1;
    return AC_OK;
}

int ac_cnn_workspace_size(int B, int H, int W, size_t* bytes) {
    if (!bytes) return fail(AC_ERR_ARG, "NULL argument");
    AC_TRY(cnn_check_shape(B, H, W));
    *bytes = cnn_train_ws_bytes(B, H, W);
    return AC_OK;
}

int ac_cnn_forward(ac_cnn* n, const uint16_t* x, int B, int H, int W, float* y, void* ws, size_t ws_bytes) {
    if (!n || !x || !y) return fail(AC_ERR_ARG, "NULL argument");
    AC_TRY(cnn_check_shape(B, H, W));
    if (!ws || ws_bytes < cnn_train_ws_bytes(B, H, W)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(n->ctx->device));
    const size_t px = static_cast<size_t>(B) * H * W;
    char* b = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(ws), 256));
    uint16_t* a1 = reinterpret_cast<uint16_t*>(b);
    uint16_t* a2 = reinterpret_cast<uint16_t*>(b + align_up(px * 32, 256));
    ProfScope ps(n->ctx, AC_K_CNN, static_cast<double>(px) * (32.0 * 5 + 8.0));
    return cnn_forward_impl(n, x, B, H, W, y, a1, a2, n->ctx->stream);
}

namespace {
// Forward pass, one loss kernel (which writes dL/dY as bf16) and the backward pass
// into n->g.  The loss scratch (px float2) shares the dZ2 buffer, which is written
// only after dY has been consumed.
template <class LossFn>
int cnn_train_pass(ac_cnn* n, const uint16_t* x, int B, int H, int W, void* ws, double* loss, float* grad_host,
                   LossFn launch_loss) {
    AC_HIP(hipSetDevice(n->ctx->device));
    hipStream_t st = n->ctx->stream;
    const size_t px = static_cast<size_t>(B) * H * W;
    const long long tiles = static_cast<long long>(B) * H * ((W + 15) / 16);
    char* b = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(ws), 256));
    const size_t a16 = align_up(px * 32, 256);
    uint16_t* A1 = reinterpret_cast<uint16_t*>(b);
    uint16_t* A2 = reinterpret_cast<uint16_t*>(b + a16);
    uint16_t* dY = reinterpret_cast<uint16_t*>(b + 2 * a16);
    uint16_t* dZ2 = reinterpret_cast<uint16_t*>(b + 3 * a16);
    uint16_t* dZ1 = reinterpret_cast<uint16_t*>(b + 4 * a16);
    float* Y = reinterpret_cast<float*>(b + 5 * a16);
    float* wpart = reinterpret_cast<float*>(b + 5 * a16 + align_up(px * 8, 256));
    float* lpart = reinterpret_cast<float*>(reinterpret_cast<char*>(wpart) +
                                            align_up(static_cast<size_t>(ac::cnn_wgrad_waves(tiles)) * 2320 * 4, 256));
    int nblk = 0;
    {
        ProfScope ps(n->ctx, AC_K_CNN, static_cast<double>(px) * (32.0 * 14 + 8.0 * 3));
        AC_TRY(cnn_forward_impl(n, x, B, H, W, Y, A1, A2, st));
        AC_HIP(launch_loss(Y, dY, reinterpret_cast<float*>(dZ2), lpart, &nblk, st));
        ac::CnnWgradArgs wa{};
        wa.B = B;
        wa.H = H;
        wa.W = W;
        wa.partial = wpart;
        wa.act = A2;
        wa.dz = dY;
        AC_HIP(ac::launch_cnn_wgrad(wa, n->g + 2 * 2320, st));
        ac::CnnConvArgs ca{};
        ca.B = B;
        ca.H = H;
        ca.W = W;
        ca.in = dY;
        ca.w = n->wb + 2 * 2304;
        ca.mask = A2;
        ca.out16 = dZ2;
        AC_HIP(ac::launch_cnn_conv(ca, st));
        wa.act = A1;
        wa.dz = dZ2;
        AC_HIP(ac::launch_cnn_wgrad(wa, n->g + 2320, st));
        ca.in = dZ2;
        ca.w = n->wb + 2304;
        ca.mask = A1;
        ca.out16 = dZ1;
        AC_HIP(ac::launch_cnn_conv(ca, st));
        wa.act = x;
        wa.dz = dZ1;
        AC_HIP(ac::launch_cnn_wgrad(wa, n->g, st));
    }
    std::vector<float> lp(nblk);
    AC_HIP(hipMemcpyAsync(lp.data(), lpart, nblk * sizeof(float), hipMemcpyDeviceToHost, st));
    if (grad_host) AC_HIP(hipMemcpyAsync(grad_host, n->g, ac::kCnnParams * sizeof(float), hipMemcpyDeviceToHost, st));
    AC_HIP(hipStreamSynchronize(st));
    double l = 0.0;
    for (float v : lp) l += v;
    if (loss) *loss = l / B;
    return AC_OK;
}
}  // namespace

int ac_cnn_grad(ac_cnn* n, const uint16_t* x, const float* t, const float* tnorm, int border, int B, int H, int W,
                void* ws, size_t ws_bytes, double* loss, float* grad_host) {
    if (!n || !x || !t || !tnorm) return fail(AC_ERR_ARG, "NULL argument");
    AC_TRY(cnn_check_shape(B, H, W));
    if (border < 0 || 2 * border >= H || 2 * border >= W) return fail(AC_ERR_ARG, "border too wide");
    if (!ws || ws_bytes < cnn_train_ws_bytes(B, H, W)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    return cnn_train_pass(n, x, B, H, W, ws, loss, grad_host,
                          [&](const float* Y, uint16_t* dY, float*, float* lpart, int* nblk, hipStream_t st) {
                              return ac::launch_cnn_loss(Y, t, tnorm, B, H, W, border, dY, lpart, nblk, st);
                          });
}

int ac_cnn_grad_residual(ac_cnn* n, const uint16_t* x, const float* rhat, const float* kappa, const float* lam,
                         const float* rnorm, int border, int B, int H, int W, void* ws, size_t ws_bytes,
                         double* loss, float* grad_host) {
    if (!n || !x || !rhat || !kappa || !lam || !rnorm) return fail(AC_ERR_ARG, "NULL argument");
    AC_TRY(cnn_check_shape(B, H, W));
    if (border < 1 || 2 * border >= H || 2 * border >= W)
        return fail(AC_ERR_ARG, "border must be at least 1 and leave an interior");
    if (!ws || ws_bytes < cnn_train_ws_bytes(B, H, W)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    return cnn_train_pass(n, x, B, H, W, ws, loss, grad_host,
                          [&](const float* Y, uint16_t* dY, float* e, float* lpart, int* nblk, hipStream_t st) {
                              return ac::launch_cnn_resloss(Y, rhat, kappa, lam, rnorm, B, H, W, border, e, dY,
                                                            lpart, nblk, st);
                          });
}

int ac_cnn_adam_step(ac_cnn* n, double lr, double beta1, double beta2, double eps) {
    if (!n) return fail(AC_ERR_ARG, "NULL argument");
    if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(AC_ERR_ARG, "invalid Adam hyper-parameters");
    AC_HIP(hipSetDevice(n->ctx->device));
    n->t += 1;
    const float bc1 = static_cast<float>(1.0 - std::pow(beta1, n->t));
    const float bc2 = static_cast<float>(1.0 - std::pow(beta2, n->t));
    AC_HIP(ac::launch_cnn_adam(n->w, n->g, n->m, n->v, static_cast<float>(lr), static_cast<float>(beta1),
                               static_cast<float>(beta2), static_cast<float>(eps), bc1, bc2, n->ctx->stream));
    AC_HIP(ac::launch_cnn_weights(n->w, n->wf, n->wb, n->bias, n->ctx->stream));
    return AC_OK;
}

int ac_cnn_make_inputs(ac_problem* p, const ac_cnn* n, int prec, const void* rhat, uint16_t* x, double* scales,
                       float* rscaled) {
    if (!p || !n || !rhat || !x) return fail(AC_ERR_ARG, "NULL argument");
    if (prec < 0 || prec > 2) return fail(AC_ERR_ARG, "unknown precision");
    AC_HIP(hipSetDevice(p->ctx->device));
    ac::CnnPrepArgs a = cnn_args(p, prec, static_cast<const char*>(rhat));
    a.c0 = n->c0;
    a.c1 = n->c1;
    SlotStats st;
    AC_TRY(slot_residuals(p, prec, a, nullptr, st));
    set_rms_scales(p, st, a, scales);
    a.x = x;
    a.rs = rscaled;
    AC_HIP(ac::launch_cnn_prep(prec, a, p->ctx->stream));
    return AC_OK;
}

int ac_problem_attach_cnn(ac_problem* p, ac_cnn* n) {
    if (!p) return fail(AC_ERR_ARG, "problem is NULL");
    if (n && n->ctx != p->ctx) return fail(AC_ERR_ARG, "network and problem belong to different contexts");
    p->cnn = n;
    return AC_OK;
}

int ac_shifted_residual(ac_problem* p, int prec, const void* rhat, const void* yhat, double* rel) {
    if (!p || !rhat || !yhat || !rel) return fail(AC_ERR_ARG, "NULL argument");
    if (prec < 0 || prec > 2) return fail(AC_ERR_ARG, "unknown precision");
    AC_HIP(hipSetDevice(p->ctx->device));
    ac::CnnPrepArgs a = cnn_args(p, prec, static_cast<const char*>(rhat));
    SlotStats st;
    AC_TRY(slot_residuals(p, prec, a, static_cast<const char*>(yhat), st));
    for (int s = 0; s < p->ns; ++s) {
        const double r = std::max(st.res(s), 0.0);
        rel[slot_to_m(p, s)] = st.rr[s] > 0 ? std::sqrt(r / st.rr[s]) : 0.0;
    }
    return AC_OK;
}

int ac_cnn_guess_workspace_size(const ac_problem* p, size_t* bytes) {
    if (!p || !bytes) return fail(AC_ERR_ARG, "NULL argument");
    *bytes = cnn_ws_bytes(p) + 256;
    return AC_OK;
}

int ac_cnn_guess(ac_problem* p, int prec, const void* rhat, void* x0hat, void* ws, size_t ws_bytes,
                 int* rejected) {
    if (!p || !rhat || !x0hat) return fail(AC_ERR_ARG, "NULL argument");
    if (!p->cnn) return fail(AC_ERR_ARG, "no warm-start network attached");
    if (prec < 0 || prec > 2) return fail(AC_ERR_ARG, "unknown precision");
    if (!ws || ws_bytes < cnn_ws_bytes(p) + 256) return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(p->ctx->device));
    char* cws = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(ws), 256));
    int fb = 0;
    AC_TRY(cnn_warm_start(p, prec, static_cast<const char*>(rhat), static_cast<char*>(x0hat), cws, &fb));
    if (rejected) *rejected = fb;
    return AC_OK;
}

int ac_cnn_set_inference(ac_cnn* n, int fused) {
    if (!n) return fail(AC_ERR_ARG, "network is NULL");
    n->fused = fused ? 1 : 0;
    return AC_OK;
}

int ac_cnn_set_guess_policy(ac_cnn* n, int scaling, double accept_ratio) {
    if (!n) return fail(AC_ERR_ARG, "network is NULL");
    if (!(accept_ratio > 0.0 && accept_ratio <= 1.0)) return fail(AC_ERR_ARG, "accept_ratio must be in (0, 1]");
    n->scaled = scaling ? 1 : 0;
    n->accept = accept_ratio;
    return AC_OK;
}
