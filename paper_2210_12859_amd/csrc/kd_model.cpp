// kd_model.cpp -- learned initial search radius: model objects, training
// driver, learned and injected-radius queries, save/load, test hooks.
//
// The model predicts y ~ ln(distance to the k-th neighbour) per query; the
// query path starts each traversal from worst0 = min(R2, fl(exp(y+m)^2)) and
// restarts, from R2, every query that found fewer than k points inside
// worst0.  Results are therefore identical to the plain traversal for any
// model; the model only affects speed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "kd_internal.h"

struct kd_model_s {
    int device = 0;
    float* d_params = nullptr;        // float32 master weights on the device
    std::vector<float> params;        // host copy
    float lo[3] = {0, 0, 0}, inv[3] = {1, 1, 1};
    float margin = 0.0f;
    int k = 0;
    std::vector<float> loss_curve;    // per-epoch mean training loss
    float holdout_rmse = 0.0f;
};

namespace kd {

namespace {

constexpr uint32_t MODEL_MAGIC = 0x4b444d31u;  // "KDM1"

// He-normal weights, zero biases, float32 (parameter order W1 b1 W2 b2 w3 b3)
std::vector<float> he_init(uint64_t seed) {
    std::vector<float> p(MLP_NPARAM, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int i = 0; i < 192; ++i) p[i] = float(nd(rng) * std::sqrt(2.0 / 3.0));
    for (int i = 256; i < 4352; ++i) p[i] = float(nd(rng) * std::sqrt(2.0 / 64.0));
    for (int i = 4416; i < 4480; ++i) p[i] = float(nd(rng) * std::sqrt(1.0 / 64.0));
    return p;
}

void norm_from_tree(kd_tree t, float lo[3], float inv[3]) {
    for (int j = 0; j < 3; ++j) {
        lo[j] = t->lo[j];
        const float ext = t->hi[j] - t->lo[j];
        inv[j] = ext > 0.0f ? 1.0f / ext : 0.0f;
    }
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes); }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

kd_status upload_params(kd_model m) {
    if (!m->d_params) KD_HIP(hipMalloc(&m->d_params, MLP_NPARAM * sizeof(float)));
    KD_HIP(hipMemcpy(m->d_params, m->params.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
    return KD_OK;
}

}  // namespace

}  // namespace kd

namespace kd {
kd_status model_view(kd_model m, MlpJob* out) {
    if (!m || !m->d_params) return set_error(KD_EINVAL, "radius model is NULL or has no parameters");
    int dev = 0;
    KD_HIP(hipGetDevice(&dev));
    if (dev != m->device) return set_error(KD_EINVAL, "radius model lives on another device");
    *out = MlpJob{};
    out->P = m->d_params;
    for (int j = 0; j < 3; ++j) {
        out->lo[j] = m->lo[j];
        out->inv[j] = m->inv[j];
    }
    out->margin = m->margin;
    return KD_OK;
}
}  // namespace kd

using namespace kd;

extern "C" {

kd_status kd_radius_model_train(kd_tree t, const float* train_q, int64_t Qt, int k, const kd_train_opts* o,
                                kd_model* out, kd_stream stream) {
    if (!out) return set_error(KD_EINVAL, "kd_radius_model_train: out is NULL");
    if (!t) return set_error(KD_EINVAL, "kd_radius_model_train: tree is NULL");
    if (t->dim != 3) return set_error(KD_EUNSUPPORTED, "kd_radius_model_train: the radius model is 3-D");
    if (t->split != KD_SPLIT_LEVEL)
        return set_error(KD_EUNSUPPORTED, "kd_radius_model_train: trees with stored split dimensions");
    if (k < 1 || k > KD_MAX_K) return set_error(KD_EINVAL, "kd_radius_model_train: k out of range [1, 64]");
    if (t->N < k) return set_error(KD_EINVAL, "kd_radius_model_train: tree has fewer than k points");
    if (Qt < 128 || Qt >= (int64_t(1) << 31)) return set_error(KD_EINVAL, "kd_radius_model_train: need 128 <= Qt < 2^31");
    if (!train_q) return set_error(KD_EINVAL, "kd_radius_model_train: train_q is NULL");
    kd_train_opts opt{20, 8192, 1e-3f, 0, 0, 0.999f};
    if (o) opt = *o;
    if (opt.epochs < 0 || opt.batch < 64 || opt.batch > (1 << 20) || !(opt.lr > 0.0f) ||
        !(opt.margin_quantile >= 0.0f && opt.margin_quantile <= 1.0f) || opt.holdout < 0)
        return set_error(KD_EINVAL, "kd_radius_model_train: bad options");
    int64_t hold = opt.holdout > 0 ? opt.holdout : std::min<int64_t>(Qt / 10, 100000);
    if (hold >= Qt) return set_error(KD_EINVAL, "kd_radius_model_train: holdout >= Qt");
    const int64_t ntrain = Qt - hold;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    try {
        std::unique_ptr<kd_model_s> m(new kd_model_s);
        KD_HIP(hipGetDevice(&m->device));
        m->k = k;
        norm_from_tree(t, m->lo, m->inv);
        m->params = he_init(opt.seed);
        kd_status s = upload_params(m.get());
        if (s != KD_OK) return s;

        // labels from the plain traversal: t = 0.5 ln(max(d2_k, 1e-14))
        DevBuf d2, idx, lab, mom, vel, part, part_loss, perm, yh, lossv;
        KD_HIP(d2.alloc(size_t(Qt) * k * sizeof(float)));
        KD_HIP(idx.alloc(size_t(Qt) * k * sizeof(int32_t)));
        KD_HIP(lab.alloc(size_t(Qt) * sizeof(float)));
        s = knn_entry(t, train_q, Qt, k, INFINITY, idx.as<int32_t>(), d2.as<float>(), nullptr, nullptr, stream,
                      "kd_radius_model_train");
        if (s != KD_OK) return s;
        KD_HIP(launch_knn_label(d2.as<float>(), k, uint32_t(Qt), lab.as<float>(), st));
        {
            // start the output bias at the mean training label, so the
            // network only has to learn the variation around it
            std::vector<float> hlab(static_cast<size_t>(ntrain));
            KD_HIP(hipMemcpyAsync(hlab.data(), lab.p, hlab.size() * sizeof(float), hipMemcpyDeviceToHost, st));
            KD_HIP(hipStreamSynchronize(st));
            double mean = 0;
            for (float v : hlab) mean += v;
            m->params[MLP_NPARAM - 1] = float(mean / double(ntrain));
            s = upload_params(m.get());
            if (s != KD_OK) return s;
        }

        const int B = opt.batch;
        const int nparts = (B + 63) / 64;
        KD_HIP(mom.alloc(MLP_NPARAM * sizeof(float)));
        KD_HIP(vel.alloc(MLP_NPARAM * sizeof(float)));
        KD_HIP(hipMemsetAsync(mom.p, 0, MLP_NPARAM * sizeof(float), st));
        KD_HIP(hipMemsetAsync(vel.p, 0, MLP_NPARAM * sizeof(float), st));
        KD_HIP(part.alloc(size_t(nparts) * MLP_NPARAM * sizeof(float)));
        KD_HIP(part_loss.alloc(size_t(nparts) * sizeof(float)));
        KD_HIP(perm.alloc(size_t(ntrain) * sizeof(uint32_t)));
        const int64_t steps_per_epoch = (ntrain + B - 1) / B;
        KD_HIP(lossv.alloc(size_t(std::max<int64_t>(1, steps_per_epoch * opt.epochs)) * sizeof(float)));

        std::vector<uint32_t> hperm(ntrain);
        int step = 0;
        for (int ep = 0; ep < opt.epochs; ++ep) {
            for (int64_t i = 0; i < ntrain; ++i) hperm[i] = uint32_t(i);
            std::mt19937_64 rng(opt.seed * 1000003ull + uint64_t(ep) + 1);
            for (int64_t i = ntrain - 1; i > 0; --i) {
                const int64_t j = int64_t(rng() % uint64_t(i + 1));
                std::swap(hperm[i], hperm[j]);
            }
            KD_HIP(hipMemcpyAsync(perm.p, hperm.data(), hperm.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
            for (int64_t b0 = 0; b0 < ntrain; b0 += B) {
                const uint32_t bs = uint32_t(std::min<int64_t>(B, ntrain - b0));
                KD_HIP(launch_mlp_fwd_bwd(m->d_params, m->lo, m->inv, train_q, lab.as<float>(), perm.as<uint32_t>(),
                                          uint32_t(b0), bs, part.as<float>(), part_loss.as<float>(), st));
                ++step;
                KD_HIP(launch_mlp_reduce_adam(part.as<float>(), part_loss.as<float>(), int((bs + 63) / 64), bs,
                                              m->d_params, mom.as<float>(), vel.as<float>(), step, opt.lr, nullptr,
                                              lossv.as<float>() + (step - 1), st));
            }
            // the pageable copy above waits for the host buffer only; keep it alive until reuse
            KD_HIP(hipStreamSynchronize(st));
        }
        std::vector<float> hl(static_cast<size_t>(step));
        if (step) KD_HIP(hipMemcpy(hl.data(), lossv.p, hl.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (int ep = 0; ep < opt.epochs; ++ep) {
            double sum = 0;
            int n = 0;
            for (int64_t i = ep * steps_per_epoch; i < (ep + 1) * steps_per_epoch && i < step; ++i, ++n) sum += hl[i];
            m->loss_curve.push_back(n ? float(sum / n) : 0.0f);
        }
        KD_HIP(hipMemcpy(m->params.data(), m->d_params, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));

        // margin: quantile of the held-out residuals t - y
        KD_HIP(yh.alloc(size_t(hold) * sizeof(float)));
        KD_HIP(launch_mlp_predict(m->d_params, m->lo, m->inv, train_q + size_t(ntrain) * 3, uint32_t(hold),
                                  yh.as<float>(), st));
        std::vector<float> hy(hold), ht(hold);
        KD_HIP(hipMemcpyAsync(hy.data(), yh.p, hold * sizeof(float), hipMemcpyDeviceToHost, st));
        KD_HIP(hipMemcpyAsync(ht.data(), lab.as<float>() + ntrain, hold * sizeof(float), hipMemcpyDeviceToHost, st));
        KD_HIP(hipStreamSynchronize(st));
        std::vector<float> res(hold);
        double se = 0;
        for (int64_t i = 0; i < hold; ++i) {
            res[i] = ht[i] - hy[i];
            se += double(res[i]) * res[i];
        }
        m->holdout_rmse = float(std::sqrt(se / double(hold)));
        std::sort(res.begin(), res.end());
        const int64_t qi = std::min<int64_t>(hold - 1, int64_t(std::floor(opt.margin_quantile * double(hold - 1) + 0.5)));
        m->margin = res[qi];
        *out = m.release();
        return KD_OK;
    } catch (const std::exception& e) {
        return set_error(KD_ENOMEM, std::string("kd_radius_model_train: ") + e.what());
    }
}

kd_status kd_model_free(kd_model m) {
    if (!m) return KD_OK;
    if (m->d_params) (void)hipFree(m->d_params);
    delete m;
    return KD_OK;
}

kd_status kd_model_info(kd_model m, int* k, float* margin, float* holdout_rmse, int* n_epochs, float* loss_curve,
                        int loss_cap) {
    if (!m) return set_error(KD_EINVAL, "kd_model_info: model is NULL");
    if (k) *k = m->k;
    if (margin) *margin = m->margin;
    if (holdout_rmse) *holdout_rmse = m->holdout_rmse;
    if (n_epochs) *n_epochs = int(m->loss_curve.size());
    if (loss_curve)
        for (int i = 0; i < loss_cap && i < int(m->loss_curve.size()); ++i) loss_curve[i] = m->loss_curve[i];
    return KD_OK;
}

kd_status kd_model_get_params(kd_model m, float* host_params, float* lo3, float* inv3) {
    if (!m) return set_error(KD_EINVAL, "kd_model_get_params: model is NULL");
    if (host_params) std::memcpy(host_params, m->params.data(), MLP_NPARAM * sizeof(float));
    if (lo3) std::memcpy(lo3, m->lo, sizeof(m->lo));
    if (inv3) std::memcpy(inv3, m->inv, sizeof(m->inv));
    return KD_OK;
}

kd_status kd_model_create(const float* host_params, const float* lo3, const float* inv3, float margin, int k,
                          kd_model* out) {
    if (!out || !host_params || !lo3 || !inv3) return set_error(KD_EINVAL, "kd_model_create: NULL argument");
    if (!std::isfinite(margin)) return set_error(KD_EINVAL, "kd_model_create: margin must be finite");
    for (int i = 0; i < MLP_NPARAM; ++i)
        if (!std::isfinite(host_params[i])) return set_error(KD_EINVAL, "kd_model_create: non-finite parameter");
    try {
        std::unique_ptr<kd_model_s> m(new kd_model_s);
        KD_HIP(hipGetDevice(&m->device));
        m->params.assign(host_params, host_params + MLP_NPARAM);
        std::memcpy(m->lo, lo3, sizeof(m->lo));
        std::memcpy(m->inv, inv3, sizeof(m->inv));
        m->margin = margin;
        m->k = k;
        kd_status s = upload_params(m.get());
        if (s != KD_OK) return s;
        *out = m.release();
        return KD_OK;
    } catch (const std::exception& e) {
        return set_error(KD_ENOMEM, std::string("kd_model_create: ") + e.what());
    }
}

kd_status kd_model_save(kd_model m, const char* path) {
    if (!m || !path) return set_error(KD_EINVAL, "kd_model_save: NULL argument");
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(KD_EINVAL, std::string("kd_model_save: cannot open ") + path);
    const uint32_t hdr[2] = {MODEL_MAGIC, uint32_t(MLP_NPARAM)};
    const int32_t k = m->k;
    const int32_t ne = int32_t(m->loss_curve.size());
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 && std::fwrite(&k, 4, 1, f) == 1 &&
              std::fwrite(&m->margin, 4, 1, f) == 1 && std::fwrite(m->lo, 4, 3, f) == 3 &&
              std::fwrite(m->inv, 4, 3, f) == 3 && std::fwrite(&m->holdout_rmse, 4, 1, f) == 1 &&
              std::fwrite(m->params.data(), 4, MLP_NPARAM, f) == size_t(MLP_NPARAM) &&
              std::fwrite(&ne, 4, 1, f) == 1 && (ne == 0 || std::fwrite(m->loss_curve.data(), 4, ne, f) == size_t(ne));
    ok = (std::fclose(f) == 0) && ok;
    return ok ? KD_OK : set_error(KD_EINVAL, "kd_model_save: write failed");
}

kd_status kd_model_load(const char* path, kd_model* out) {
    if (!path || !out) return set_error(KD_EINVAL, "kd_model_load: NULL argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(KD_EINVAL, std::string("kd_model_load: cannot open ") + path);
    uint32_t hdr[2] = {0, 0};
    int32_t k = 0, ne = 0;
    float margin = 0, lo[3], inv[3], rmse = 0;
    std::vector<float> p(MLP_NPARAM);
    bool ok = std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == MODEL_MAGIC && hdr[1] == uint32_t(MLP_NPARAM) &&
              std::fread(&k, 4, 1, f) == 1 && std::fread(&margin, 4, 1, f) == 1 && std::fread(lo, 4, 3, f) == 3 &&
              std::fread(inv, 4, 3, f) == 3 && std::fread(&rmse, 4, 1, f) == 1 &&
              std::fread(p.data(), 4, MLP_NPARAM, f) == size_t(MLP_NPARAM) && std::fread(&ne, 4, 1, f) == 1 &&
              ne >= 0 && ne < (1 << 20);
    std::vector<float> curve(ok ? size_t(ne) : 0);
    if (ok && ne > 0) ok = std::fread(curve.data(), 4, ne, f) == size_t(ne);
    std::fclose(f);
    if (!ok) return set_error(KD_EINVAL, "kd_model_load: not a model file or truncated");
    kd_status s = kd_model_create(p.data(), lo, inv, margin, k, out);
    if (s != KD_OK) return s;
    (*out)->holdout_rmse = rmse;
    (*out)->loss_curve = curve;
    return KD_OK;
}

kd_status kd_knn_learned(kd_tree t, kd_model m, const float* queries, int64_t Q, int k, float maxRadius,
                         int32_t* out_idx, float* out_d2, uint32_t* visited, kd_stats* stats, const kd_opts* opts,
                         kd_stream stream) {
    kd_status s = check_query_args_public(t, queries, Q, k, maxRadius, out_idx, "kd_knn_learned");
    if (s != KD_OK) return s;
    if (!m) return set_error(KD_EINVAL, "kd_knn_learned: model is NULL");
    if (t->dim != 3) return set_error(KD_EUNSUPPORTED, "kd_knn_learned: the radius model is 3-D");
    if (t->split != KD_SPLIT_LEVEL)
        return set_error(KD_EUNSUPPORTED, "kd_knn_learned: trees with stored split dimensions");
    if (stats) *stats = kd_stats{0, 0, 0, 0, 0.0f, 0.0f, 0.0f, 0.0f};
    if (Q == 0 || t->N == 0)
        return knn_entry(t, queries, Q, k, maxRadius, out_idx, out_d2, visited, opts, stream, "kd_knn_learned");
    QueryPlan plan;
    s = resolve_plan_public(t, k, maxRadius, opts, plan);
    if (s != KD_OK) return s;
    LearnedSpec ls{};
    ls.params = m->d_params;
    std::memcpy(ls.lo, m->lo, sizeof(ls.lo));
    std::memcpy(ls.inv, m->inv, sizeof(ls.inv));
    ls.margin = m->margin;
    return run_knn(t, queries, Q, plan, out_idx, out_d2, visited, stream, &ls, stats);
}

kd_status kd_knn_with_radius(kd_tree t, const float* r0, const float* queries, int64_t Q, int k, float maxRadius,
                             int32_t* out_idx, float* out_d2, uint32_t* visited, uint8_t* fell_back,
                             const kd_opts* opts, kd_stream stream) {
    kd_status s = check_query_args_public(t, queries, Q, k, maxRadius, out_idx, "kd_knn_with_radius");
    if (s != KD_OK) return s;
    if (Q > 0 && !r0) return set_error(KD_EINVAL, "kd_knn_with_radius: r0 is NULL");
    if (t->split != KD_SPLIT_LEVEL)
        return set_error(KD_EUNSUPPORTED, "kd_knn_with_radius: trees with stored split dimensions");
    if (Q == 0 || t->N == 0) {
        s = knn_entry(t, queries, Q, k, maxRadius, out_idx, out_d2, visited, opts, stream, "kd_knn_with_radius");
        if (s == KD_OK && fell_back && Q > 0)
            KD_HIP(hipMemsetAsync(fell_back, 0, size_t(Q), reinterpret_cast<hipStream_t>(stream)));
        return s;
    }
    QueryPlan plan;
    s = resolve_plan_public(t, k, maxRadius, opts, plan);
    if (s != KD_OK) return s;
    LearnedSpec ls{};
    ls.r0 = r0;
    ls.fb_flag = fell_back;
    return run_knn(t, queries, Q, plan, out_idx, out_d2, visited, stream, &ls, nullptr);
}

kd_status kd_mlp_predict(kd_model m, const float* queries, int64_t n, float* y, kd_stream stream) {
    if (!m) return set_error(KD_EINVAL, "kd_mlp_predict: model is NULL");
    if (n < 0 || n >= (int64_t(1) << 31)) return set_error(KD_EINVAL, "kd_mlp_predict: n out of range");
    if (n > 0 && (!queries || !y)) return set_error(KD_EINVAL, "kd_mlp_predict: NULL pointer");
    KD_HIP(launch_mlp_predict(m->d_params, m->lo, m->inv, queries, uint32_t(n), y,
                              reinterpret_cast<hipStream_t>(stream)));
    return KD_OK;
}

kd_status kd_mlp_grad(kd_model m, const float* queries, const float* targets, int64_t n, float* host_grad,
                      float* host_loss, kd_stream stream) {
    if (!m) return set_error(KD_EINVAL, "kd_mlp_grad: model is NULL");
    if (n < 1 || n > (1 << 20)) return set_error(KD_EINVAL, "kd_mlp_grad: n out of range [1, 2^20]");
    if (!queries || !targets || !host_grad) return set_error(KD_EINVAL, "kd_mlp_grad: NULL pointer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    try {
        const int nparts = int((n + 63) / 64);
        DevBuf part, part_loss, grad, loss;
        KD_HIP(part.alloc(size_t(nparts) * MLP_NPARAM * sizeof(float)));
        KD_HIP(part_loss.alloc(size_t(nparts) * sizeof(float)));
        KD_HIP(grad.alloc(MLP_NPARAM * sizeof(float)));
        KD_HIP(loss.alloc(sizeof(float)));
        KD_HIP(launch_mlp_fwd_bwd(m->d_params, m->lo, m->inv, queries, targets, nullptr, 0, uint32_t(n),
                                  part.as<float>(), part_loss.as<float>(), st));
        KD_HIP(launch_mlp_reduce_adam(part.as<float>(), part_loss.as<float>(), nparts, uint32_t(n), m->d_params,
                                      nullptr, nullptr, 0, 0.0f, grad.as<float>(), loss.as<float>(), st));
        KD_HIP(hipMemcpyAsync(host_grad, grad.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
        float hl = 0;
        KD_HIP(hipMemcpyAsync(&hl, loss.p, sizeof(float), hipMemcpyDeviceToHost, st));
        KD_HIP(hipStreamSynchronize(st));
        if (host_loss) *host_loss = hl;
        return KD_OK;
    } catch (const std::exception& e) {
        return set_error(KD_ENOMEM, std::string("kd_mlp_grad: ") + e.what());
    }
}

kd_status kd_mlp_worst0(kd_model m, const float* queries, int64_t n, float maxRadius, float* worst0,
                        kd_stream stream) {
    if (!m) return set_error(KD_EINVAL, "kd_mlp_worst0: model is NULL");
    if (n < 0 || n >= (int64_t(1) << 31)) return set_error(KD_EINVAL, "kd_mlp_worst0: n out of range");
    if (std::isnan(maxRadius) || maxRadius < 0.0f)
        return set_error(KD_EINVAL, "kd_mlp_worst0: maxRadius must be >= 0 (or +inf)");
    if (n == 0) return KD_OK;
    if (!queries || !worst0) return set_error(KD_EINVAL, "kd_mlp_worst0: NULL pointer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float R2 = maxRadius * maxRadius;
    try {
        DevBuf recs;
        KD_HIP(recs.alloc(size_t(n) * 16));
        KD_HIP(launch_mlp_worst0_rows(m->d_params, m->lo, m->inv, m->margin, R2, queries, uint32_t(n), recs.p, worst0,
                                      st));
        // the records are freed on return
        KD_HIP(hipStreamSynchronize(st));
        return KD_OK;
    } catch (const std::exception& e) {
        return set_error(KD_ENOMEM, std::string("kd_mlp_worst0: ") + e.what());
    }
}

kd_status kd_mlp_train_step(kd_model m, const float* queries, const float* targets, int64_t n, int step, float lr,
                            float* host_m, float* host_v, float* host_grad, float* host_loss, kd_stream stream) {
    if (!m) return set_error(KD_EINVAL, "kd_mlp_train_step: model is NULL");
    if (n < 1 || n > (1 << 20)) return set_error(KD_EINVAL, "kd_mlp_train_step: n out of range [1, 2^20]");
    if (step < 1) return set_error(KD_EINVAL, "kd_mlp_train_step: step counts from 1");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return set_error(KD_EINVAL, "kd_mlp_train_step: lr must be > 0");
    if (!queries || !targets || !host_m || !host_v) return set_error(KD_EINVAL, "kd_mlp_train_step: NULL pointer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    try {
        const int nparts = int((n + 63) / 64);
        DevBuf part, part_loss, grad, loss, mom, vel;
        KD_HIP(part.alloc(size_t(nparts) * MLP_NPARAM * sizeof(float)));
        KD_HIP(part_loss.alloc(size_t(nparts) * sizeof(float)));
        KD_HIP(grad.alloc(MLP_NPARAM * sizeof(float)));
        KD_HIP(loss.alloc(sizeof(float)));
        KD_HIP(mom.alloc(MLP_NPARAM * sizeof(float)));
        KD_HIP(vel.alloc(MLP_NPARAM * sizeof(float)));
        KD_HIP(hipMemcpyAsync(mom.p, host_m, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st));
        KD_HIP(hipMemcpyAsync(vel.p, host_v, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st));
        KD_HIP(launch_mlp_fwd_bwd(m->d_params, m->lo, m->inv, queries, targets, nullptr, 0, uint32_t(n),
                                  part.as<float>(), part_loss.as<float>(), st));
        KD_HIP(launch_mlp_reduce_adam(part.as<float>(), part_loss.as<float>(), nparts, uint32_t(n), m->d_params,
                                      mom.as<float>(), vel.as<float>(), step, lr, grad.as<float>(), loss.as<float>(),
                                      st));
        KD_HIP(hipMemcpyAsync(host_m, mom.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
        KD_HIP(hipMemcpyAsync(host_v, vel.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
        if (host_grad) KD_HIP(hipMemcpyAsync(host_grad, grad.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
        float hl = 0;
        KD_HIP(hipMemcpyAsync(&hl, loss.p, sizeof(float), hipMemcpyDeviceToHost, st));
        KD_HIP(hipMemcpyAsync(m->params.data(), m->d_params, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
        KD_HIP(hipStreamSynchronize(st));
        if (host_loss) *host_loss = hl;
        return KD_OK;
    } catch (const std::exception& e) {
        return set_error(KD_ENOMEM, std::string("kd_mlp_train_step: ") + e.what());
    }
}

}  // extern "C"
