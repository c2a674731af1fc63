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
    float* d_x = nullptr;        // lx_phi_leja_learned: features [n][8]
    float* d_y = nullptr;        // and predictions [n][2] (device) ...
    float* h_y = nullptr;        // ... copied to pinned host memory
    size_t xy_cap = 0;
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
    (void)hipFree(p->d_x);
    (void)hipFree(p->d_y);
    (void)hipHostFree(p->h_y);
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
        if ((q.op.kind != LX_OP_DIFFADV2D && q.op.kind != LX_OP_BURGERS2D) || q.op.nx < 1 || q.op.ny < 1 ||
            !(q.op.dx > 0.0) || !(q.h > 0.0) || q.d_v == nullptr ||
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

lx_status lx_phi_leja_learned(lx_ctx* ctx, lx_predictor* p, int n, const lx_instance* inst, double margin_log_rho,
                              double margin_log_sweeps, int power_iters, double safety, const lx_leja_opts* o,
                              lx_instance_result* res, int* fallbacks) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    if (p == nullptr || p->ctx != ctx) return lx_internal_fail(ctx, LX_EINVAL, "the predictor belongs to another context");
    if (n < 1 || n > 65536 || inst == nullptr || res == nullptr)
        return lx_internal_fail(ctx, LX_EINVAL, "batch of %d instances (1..65536) with inputs and results", n);
    if (!std::isfinite(margin_log_rho) || !std::isfinite(margin_log_sweeps) || margin_log_rho < 0.0 ||
        margin_log_sweeps < 0.0)
        return lx_internal_fail(ctx, LX_EINVAL, "margins must be finite and >= 0");
    if (power_iters < 1 || power_iters > LX_MAX_ITERS || !(safety > 0.0) || !std::isfinite(safety))
        return lx_internal_fail(ctx, LX_EINVAL, "the fallback needs 1..%d power iterations and a safety > 0",
                                LX_MAX_ITERS);
    lx_leja_opts opt{1e-8, 0.0, 500, 1e4};
    if (o != nullptr) opt = *o;
    if (opt.max_iters < 1 || opt.max_iters > LX_MAX_ITERS)
        return lx_internal_fail(ctx, LX_EINVAL, "max_iters %d outside 1..%d", opt.max_iters, LX_MAX_ITERS);

    // ---- predictions ----
    const size_t nn = static_cast<size_t>(n);
    if (nn > p->xy_cap) {
        LXP_HIP(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(p->d_x);
        (void)hipFree(p->d_y);
        (void)hipHostFree(p->h_y);
        p->d_x = p->d_y = p->h_y = nullptr;
        p->xy_cap = 0;
        if (hipMalloc(&p->d_x, sizeof(float) * 8 * nn) != hipSuccess ||
            hipMalloc(&p->d_y, sizeof(float) * 2 * nn) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&p->h_y), sizeof(float) * 2 * nn, hipHostMallocDefault) != hipSuccess)
            return lx_internal_fail(ctx, LX_ENOMEM, "prediction buffers for %d instances", n);
        p->xy_cap = nn;
    }
    lx_status s = lx_instance_features(ctx, n, inst, p->d_x);
    if (s != LX_OK) return s;
    s = lx_predictor_infer(p, p->d_x, n, p->d_y);
    if (s != LX_OK) return s;
    LXP_HIP(ctx, hipMemcpyAsync(p->h_y, p->d_y, sizeof(float) * 2 * nn, hipMemcpyDeviceToHost, ctx->stream));
    LXP_HIP(ctx, hipStreamSynchronize(ctx->stream));

    // ---- the learned batch: predicted shift, scale and budget ----
    std::vector<lx_instance> q;
    std::vector<int> idx, fb;
    q.reserve(nn);
    idx.reserve(nn);
    for (int i = 0; i < n; ++i) {
        const double a = p->h_y[2 * i], b = p->h_y[2 * i + 1];
        const double lam = -std::exp(a + margin_log_rho);
        const double sweeps = std::ceil(std::exp(b + margin_log_sweeps)) + 1.0;
        res[i] = lx_instance_result{};
        if (!std::isfinite(lam) || !(lam < 0.0) || !std::isfinite(sweeps)) {
            fb.push_back(i);
            continue;
        }
        lx_instance r = inst[i];
        r.c = lam / 2.0;
        r.gamma = -lam / 4.0;
        r.budget = static_cast<int>(std::min(static_cast<double>(opt.max_iters), std::max(1.0, sweeps)));
        q.push_back(r);
        idx.push_back(i);
    }
    lx_stats acc{};
    if (!q.empty()) {
        std::vector<lx_instance_result> r(q.size());
        s = lx_phi_leja_batched(ctx, static_cast<int>(q.size()), q.data(), 0, 1.0, &opt, r.data());
        if (s != LX_OK && s != LX_ENOTCONV && s != LX_ENONFINITE) return s;
        acc = ctx->stats;
        for (size_t k = 0; k < q.size(); ++k) {
            res[idx[k]] = r[k];
            if (r[k].status != LX_OK) fb.push_back(idx[k]);
        }
    }
    // ---- the plain method for the rest ----
    lx_status worst = LX_OK;
    if (!fb.empty()) {
        std::sort(fb.begin(), fb.end());
        std::vector<lx_instance> qf;
        qf.reserve(fb.size());
        for (int i : fb) {
            lx_instance r = inst[i];
            r.budget = 0;
            qf.push_back(r);
        }
        std::vector<lx_instance_result> r(fb.size());
        s = lx_phi_leja_batched(ctx, static_cast<int>(fb.size()), qf.data(), power_iters, safety, &opt, r.data());
        if (s != LX_OK && s != LX_ENOTCONV && s != LX_ENONFINITE) return s;
        for (size_t k = 0; k < fb.size(); ++k) {
            res[fb[k]] = r[k];
            res[fb[k]].fallback = 1;
        }
        const lx_stats& f = ctx->stats;
        acc.n_apply = std::max(acc.n_apply, f.n_apply);
        acc.bytes += f.bytes;
        acc.plan_ms += f.plan_ms;
        acc.loop_ms += f.loop_ms;
        acc.sweep_ms += f.sweep_ms;
        acc.depth = f.depth;
    }
    for (int i = 0; i < n; ++i) {
        if (res[i].status == LX_ENONFINITE || res[i].status == LX_EDEVICE) worst = static_cast<lx_status>(res[i].status);
        else if (res[i].status == LX_ENOTCONV && worst == LX_OK) worst = LX_ENOTCONV;
    }
    acc.status = worst;
    ctx->stats = acc;
    if (fallbacks != nullptr) *fallbacks = static_cast<int>(fb.size());
    if (worst != LX_OK) return lx_internal_fail(ctx, worst, "at least one instance failed after its fallback");
    return LX_OK;
}

}  // extern "C"
