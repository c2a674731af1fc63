// C ABI of the spectral/budget predictor (declarations and contracts in lx.h).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lx.h"
#include "lx_ctx.h"
#include "mlp_device.h"

struct lx_predictor {
    lx_ctx* ctx = nullptr;
    float* theta = nullptr;      // parameters, then Adam moments m and v (3 * kMlpParams)
    float* grad = nullptr;
    double* d_loss = nullptr;
    float* scratch = nullptr;
    size_t scratch_rows = 0;
    int* d_idx = nullptr;
    size_t idx_cap = 0;
    double* h_loss = nullptr;    // pinned
    lx::MlpScaling sc{};
    int t = 0;                   // Adam steps taken
};

namespace {

#define LXP_HIP(ctx, call)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return lx_internal_fail((ctx), LX_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014)
uint64_t splitmix_next(uint64_t* state) {
    uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

double unit(uint64_t* state) { return static_cast<double>(splitmix_next(state) >> 11) * 0x1.0p-53; }

lx_status grow_scratch(lx_predictor* p, size_t rows) {
    if (rows <= p->scratch_rows) return LX_OK;
    (void)hipStreamSynchronize(p->ctx->stream);
    (void)hipFree(p->scratch);
    p->scratch = nullptr;
    p->scratch_rows = 0;
    if (hipMalloc(&p->scratch, sizeof(float) * rows * lx::kMlpRow) != hipSuccess)
        return lx_internal_fail(p->ctx, LX_ENOMEM, "predictor scratch for %zu samples", rows);
    p->scratch_rows = rows;
    return LX_OK;
}

lx_status grow_idx(lx_predictor* p, size_t n) {
    if (n <= p->idx_cap) return LX_OK;
    (void)hipStreamSynchronize(p->ctx->stream);
    (void)hipFree(p->d_idx);
    p->d_idx = nullptr;
    p->idx_cap = 0;
    if (hipMalloc(&p->d_idx, sizeof(int) * n) != hipSuccess)
        return lx_internal_fail(p->ctx, LX_ENOMEM, "minibatch index list of %zu entries", n);
    p->idx_cap = n;
    return LX_OK;
}

}  // namespace

extern "C" {

int lx_predictor_state_size(void) { return LX_MLP_STATE; }

lx_status lx_predictor_create(lx_ctx* ctx, unsigned long long seed, lx_predictor** out) {
    if (ctx == nullptr || out == nullptr) return LX_EINVAL;
    *out = nullptr;
    lx_predictor* p = new lx_predictor();
    p->ctx = ctx;
    auto bail = [&](lx_status s) {
        lx_predictor_destroy(p);
        return s;
    };
    if (hipMalloc(&p->theta, sizeof(float) * 3 * lx::kMlpParams) != hipSuccess ||
        hipMalloc(&p->grad, sizeof(float) * lx::kMlpParams) != hipSuccess ||
        hipMalloc(&p->d_loss, sizeof(double)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&p->h_loss), sizeof(double), hipHostMallocDefault) != hipSuccess)
        return bail(LX_ENOMEM);
    // He-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)), zero biases and moments
    std::vector<float> h(3 * static_cast<size_t>(lx::kMlpParams), 0.0f);
    uint64_t st = seed;
    auto fill = [&](int off, int count, int fan_in) {
        const double a = std::sqrt(6.0 / fan_in);
        for (int i = 0; i < count; ++i) h[static_cast<size_t>(off + i)] = static_cast<float>((2.0 * unit(&st) - 1.0) * a);
    };
    fill(lx::kPW1, lx::kMlpH * lx::kMlpIn, lx::kMlpIn);
    fill(lx::kPW2, lx::kMlpH * lx::kMlpH, lx::kMlpH);
    fill(lx::kPW3, lx::kMlpOut * lx::kMlpH, lx::kMlpH);
    if (hipMemcpy(p->theta, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bail(LX_EDEVICE);
    for (int j = 0; j < lx::kMlpIn; ++j) p->sc.std_x[j] = 1.0f;
    for (int o = 0; o < lx::kMlpOut; ++o) p->sc.std_y[o] = 1.0f;
    ctx->predictors.push_back(p);
    *out = p;
    return LX_OK;
}

void lx_predictor_destroy(lx_predictor* p) {
    if (p == nullptr) return;
    if (p->ctx) {
        auto& v = p->ctx->predictors;
        v.erase(std::remove(v.begin(), v.end(), p), v.end());
        (void)hipStreamSynchronize(p->ctx->stream);
    }
    (void)hipFree(p->theta);
    (void)hipFree(p->grad);
    (void)hipFree(p->d_loss);
    (void)hipFree(p->scratch);
    (void)hipFree(p->d_idx);
    (void)hipHostFree(p->h_loss);
    delete p;
}

lx_status lx_predictor_set_scaling(lx_predictor* p, const float* mean_x, const float* std_x, const float* mean_y,
                                   const float* std_y) {
    if (p == nullptr || mean_x == nullptr || std_x == nullptr || mean_y == nullptr || std_y == nullptr)
        return LX_EINVAL;
    for (int j = 0; j < lx::kMlpIn; ++j)
        if (!(std_x[j] > 0.0f) || !std::isfinite(mean_x[j])) return lx_internal_fail(p->ctx, LX_EINVAL, "input scaling");
    for (int o = 0; o < lx::kMlpOut; ++o)
        if (!(std_y[o] > 0.0f) || !std::isfinite(mean_y[o])) return lx_internal_fail(p->ctx, LX_EINVAL, "target scaling");
    std::memcpy(p->sc.mean_x, mean_x, sizeof(p->sc.mean_x));
    std::memcpy(p->sc.std_x, std_x, sizeof(p->sc.std_x));
    std::memcpy(p->sc.mean_y, mean_y, sizeof(p->sc.mean_y));
    std::memcpy(p->sc.std_y, std_y, sizeof(p->sc.std_y));
    return LX_OK;
}

lx_status lx_predictor_get_state(const lx_predictor* p, float* state) {
    if (p == nullptr || state == nullptr) return LX_EINVAL;
    if (hipStreamSynchronize(p->ctx->stream) != hipSuccess ||
        hipMemcpy(state, p->theta, sizeof(float) * 3 * lx::kMlpParams, hipMemcpyDeviceToHost) != hipSuccess)
        return LX_EDEVICE;
    float* s = state + 3 * lx::kMlpParams;
    std::memcpy(s, &p->sc, sizeof(lx::MlpScaling));
    s[sizeof(lx::MlpScaling) / sizeof(float)] = static_cast<float>(p->t);
    return LX_OK;
}

lx_status lx_predictor_set_state(lx_predictor* p, const float* state) {
    if (p == nullptr || state == nullptr) return LX_EINVAL;
    const float* s = state + 3 * lx::kMlpParams;
    lx::MlpScaling sc;
    std::memcpy(&sc, s, sizeof(sc));
    const lx_status st = lx_predictor_set_scaling(p, sc.mean_x, sc.std_x, sc.mean_y, sc.std_y);
    if (st != LX_OK) return st;
    const float t = s[sizeof(lx::MlpScaling) / sizeof(float)];
    if (!(t >= 0.0f) || t > 1e9f) return lx_internal_fail(p->ctx, LX_EINVAL, "bad step count in state");
    p->t = static_cast<int>(t);
    LXP_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    LXP_HIP(p->ctx, hipMemcpy(p->theta, state, sizeof(float) * 3 * lx::kMlpParams, hipMemcpyHostToDevice));
    return LX_OK;
}

lx_status lx_predictor_save(const lx_predictor* p, const char* path) {
    if (p == nullptr || path == nullptr) return LX_EINVAL;
    std::vector<float> s(LX_MLP_STATE);
    lx_status st = lx_predictor_get_state(p, s.data());
    if (st != LX_OK) return st;
    FILE* f = std::fopen(path, "wb");
    if (f == nullptr) return lx_internal_fail(p->ctx, LX_EINVAL, "cannot write %s", path);
    const char magic[8] = {'L', 'X', 'M', 'L', 'P', '0', '0', '1'};
    const int32_t n = LX_MLP_STATE;
    const bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&n, sizeof(n), 1, f) == 1 &&
                    std::fwrite(s.data(), sizeof(float), s.size(), f) == s.size();
    std::fclose(f);
    return ok ? LX_OK : lx_internal_fail(p->ctx, LX_EINVAL, "short write to %s", path);
}

lx_status lx_predictor_load(lx_predictor* p, const char* path) {
    if (p == nullptr || path == nullptr) return LX_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (f == nullptr) return lx_internal_fail(p->ctx, LX_EINVAL, "cannot read %s", path);
    char magic[8];
    int32_t n = 0;
    std::vector<float> s(LX_MLP_STATE);
    const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "LXMLP001", 8) == 0 &&
                    std::fread(&n, sizeof(n), 1, f) == 1 && n == LX_MLP_STATE &&
                    std::fread(s.data(), sizeof(float), s.size(), f) == s.size();
    std::fclose(f);
    if (!ok) return lx_internal_fail(p->ctx, LX_EINVAL, "%s is not a predictor state file", path);
    return lx_predictor_set_state(p, s.data());
}

lx_status lx_predictor_gradient(lx_predictor* p, const float* d_x, const float* d_y, int n, float* grad,
                                double* loss) {
    if (p == nullptr || d_x == nullptr || d_y == nullptr || n < 1) return LX_EINVAL;
    lx_ctx* ctx = p->ctx;
    lx_status s = grow_scratch(p, static_cast<size_t>(n));
    if (s != LX_OK) return s;
    LXP_HIP(ctx, lx::launch_mlp_fwd_bwd(p->theta, d_x, d_y, nullptr, n, p->sc, p->scratch, ctx->stream));
    LXP_HIP(ctx, lx::launch_mlp_grad(p->scratch, n, p->grad, p->d_loss, ctx->stream));
    LXP_HIP(ctx, hipMemcpyAsync(p->h_loss, p->d_loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (grad != nullptr)
        LXP_HIP(ctx, hipMemcpyAsync(grad, p->grad, sizeof(float) * lx::kMlpParams, hipMemcpyDeviceToHost, ctx->stream));
    LXP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (loss) *loss = *p->h_loss;
    return LX_OK;
}

lx_status lx_predictor_train(lx_predictor* p, const float* d_x, const float* d_y, int n, int steps, int batch,
                             float lr, unsigned long long seed, const int* order, double* final_loss) {
    if (p == nullptr || d_x == nullptr || d_y == nullptr || n < 1 || steps < 1 || batch < 1 || batch > n ||
        !(lr > 0.0f))
        return p ? lx_internal_fail(p->ctx, LX_EINVAL, "train: n %d steps %d batch %d lr %g", n, steps, batch, lr)
                 : LX_EINVAL;
    lx_ctx* ctx = p->ctx;
    const size_t total = static_cast<size_t>(steps) * batch;
    lx_status s = grow_scratch(p, static_cast<size_t>(batch));
    if (s == LX_OK) s = grow_idx(p, total);
    if (s != LX_OK) return s;
    std::vector<int> idx(total);
    if (order != nullptr) {
        for (size_t i = 0; i < total; ++i) {
            if (order[i] < 0 || order[i] >= n) return lx_internal_fail(ctx, LX_EINVAL, "order[%zu] out of range", i);
            idx[i] = order[i];
        }
    } else {
        // epochs of a Fisher-Yates shuffle driven by splitmix64
        std::vector<int> perm(static_cast<size_t>(n));
        uint64_t st = seed;
        size_t pos = static_cast<size_t>(n);
        for (size_t i = 0; i < total; ++i) {
            if (pos == static_cast<size_t>(n)) {
                for (int k = 0; k < n; ++k) perm[static_cast<size_t>(k)] = k;
                for (int k = n - 1; k > 0; --k) {
                    const int r = static_cast<int>(splitmix_next(&st) % static_cast<uint64_t>(k + 1));
                    std::swap(perm[static_cast<size_t>(k)], perm[static_cast<size_t>(r)]);
                }
                pos = 0;
            }
            idx[i] = perm[pos++];
        }
    }
    LXP_HIP(ctx, hipMemcpyAsync(p->d_idx, idx.data(), sizeof(int) * total, hipMemcpyHostToDevice, ctx->stream));
    for (int k = 0; k < steps; ++k) {
        LXP_HIP(ctx, lx::launch_mlp_fwd_bwd(p->theta, d_x, d_y, p->d_idx + static_cast<size_t>(k) * batch, batch, p->sc,
                                            p->scratch, ctx->stream));
        LXP_HIP(ctx, lx::launch_mlp_grad(p->scratch, batch, p->grad, k + 1 == steps ? p->d_loss : nullptr, ctx->stream));
        p->t += 1;
        LXP_HIP(ctx, lx::launch_mlp_adam(p->theta, p->grad, p->theta + lx::kMlpParams, p->theta + 2 * lx::kMlpParams,
                                         p->t, lr, ctx->stream));
    }
    LXP_HIP(ctx, hipMemcpyAsync(p->h_loss, p->d_loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    LXP_HIP(ctx, hipStreamSynchronize(ctx->stream));   // idx (host vector) must outlive the copy
    if (final_loss) *final_loss = *p->h_loss;
    return LX_OK;
}

lx_status lx_predictor_infer(lx_predictor* p, const float* d_x, int n, float* d_y) {
    if (p == nullptr || d_x == nullptr || d_y == nullptr || n < 1) return LX_EINVAL;
    LXP_HIP(p->ctx, lx::launch_mlp_infer(p->theta, d_x, n, p->sc, d_y, p->ctx->stream));
    return LX_OK;
}

lx_status lx_instance_features(lx_ctx* ctx, int n, const lx_instance* inst, float* d_x) {
    if (ctx == nullptr || inst == nullptr || d_x == nullptr || n < 1) return LX_EINVAL;
    std::vector<lx::FeatureInst> f(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        const lx_instance& q = inst[i];
        if (q.op.nx < 1 || q.op.ny < 1 || !(q.op.dx > 0.0) || !(q.h > 0.0) || q.d_v == nullptr ||
            (q.op.kind == LX_OP_BURGERS2D && (q.d_u == nullptr || !(q.op.nu > 0.0))) ||
            (q.op.kind == LX_OP_DIFFADV2D && !(q.op.D > 0.0)))
            return lx_internal_fail(ctx, LX_EINVAL, "features: instance %d", i);
        lx::FeatureInst& g = f[static_cast<size_t>(i)];
        g.nx = q.op.nx;
        g.ny = q.op.ny;
        g.l = q.l;
        g.burgers = q.op.kind == LX_OP_BURGERS2D;
        g.dx = q.op.dx;
        g.h = q.h;
        g.D = g.burgers ? q.op.nu : q.op.D;
        g.vx = q.op.vx;
        g.vy = q.op.vy;
        g.u = g.burgers ? q.d_u : q.d_v;
    }
    lx_batch_ws& W = ctx->batch;
    const size_t bytes = sizeof(lx::FeatureInst) * f.size();
    if (bytes > W.cap_feat) {
        LXP_HIP(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(W.d_feat);
        (void)hipHostFree(W.h_feat);
        W.d_feat = W.h_feat = nullptr;
        W.cap_feat = 0;
        if (hipMalloc(&W.d_feat, bytes) != hipSuccess || hipHostMalloc(&W.h_feat, bytes, hipHostMallocDefault) != hipSuccess)
            return lx_internal_fail(ctx, LX_ENOMEM, "feature descriptors");
        W.cap_feat = bytes;
    }
    LXP_HIP(ctx, hipStreamSynchronize(ctx->stream));   // the pinned staging may still feed an earlier copy
    std::memcpy(W.h_feat, f.data(), bytes);
    LXP_HIP(ctx, hipMemcpyAsync(W.d_feat, W.h_feat, bytes, hipMemcpyHostToDevice, ctx->stream));
    LXP_HIP(ctx, lx::launch_features(static_cast<const lx::FeatureInst*>(W.d_feat), n, d_x, ctx->stream));
    return LX_OK;
}

}  // extern "C"
