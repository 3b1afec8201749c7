// kd_autotune.cpp -- picks launch options for a tree and k by timing them.
//
// Candidates: workgroup size x persistent waves per CU x Morton sort bits.
// Every candidate returns byte-identical results (the options only change
// which lane serves which query and in what order), so the choice is purely
// a matter of speed.  The winner is kept on the tree per compiled list size
// K and used by kd_knn / kd_knn_ex / kd_knn_learned when called with default
// options.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "kd_internal.h"

namespace kd {

bool tuned_opts(kd_tree t, int K, kd_opts* out) {
    std::lock_guard<std::mutex> lk(t->tune_mu);
    for (const auto& e : t->tuned)
        if (e.k_template == K) {
            *out = e.opts;
            return true;
        }
    return false;
}

void set_tuned(kd_tree t, int K, const kd_opts& o) {
    std::lock_guard<std::mutex> lk(t->tune_mu);
    for (auto& e : t->tuned)
        if (e.k_template == K) {
            e.opts = o;
            return;
        }
    t->tuned.push_back(TuneEntry{K, o});
}

}  // namespace kd

using namespace kd;

extern "C" {

kd_status kd_autotune(kd_tree t, const float* sample_q, int64_t Qs, int k, float maxRadius, kd_opts* best_out,
                      float* best_ms, kd_stream stream) {
    if (!t) return set_error(KD_EINVAL, "kd_autotune: tree is NULL");
    if (k < 1 || k > KD_MAX_K) return set_error(KD_EINVAL, "kd_autotune: k out of range [1, 64]");
    if (Qs < 1 || Qs >= (int64_t(1) << 31)) return set_error(KD_EINVAL, "kd_autotune: Qs out of range");
    if (!sample_q) return set_error(KD_EINVAL, "kd_autotune: sample_q is NULL");
    if (std::isnan(maxRadius) || maxRadius < 0.0f) return set_error(KD_EINVAL, "kd_autotune: bad maxRadius");
    if (t->N == 0) return set_error(KD_EINVAL, "kd_autotune: empty tree");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int K = k_template(k);
    std::vector<kd_opts> cands;
    const int blocks[] = {256, 512, 1024};
    const int waves[] = {8, 12, 16, 24, 32};
    const int sorts[] = {0, 16, 24, 32};
    const int prunes[] = {1, 2};
    const int ldsl[] = {0, 10};  // top levels in LDS (dim 4: 32 KB of records)
    for (int b : blocks) {
        if (K >= 32 && b > 256) continue;
        for (int w : waves)
            for (int sb : sorts)
                for (int pr : prunes)
                    for (int l : ldsl)
                        if (l == 0 || !t->d_dims)  // stored dimensions: nodes from global memory
                            cands.push_back(kd_opts{b, l, sb, w, 0, pr});
    }
    int32_t* idx = nullptr;
    float* d2 = nullptr;
    unsigned long long* d_sum = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (idx) (void)hipFree(idx);
        if (d2) (void)hipFree(d2);
        if (d_sum) (void)hipFree(d_sum);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e = hipMalloc(&idx, size_t(Qs) * k * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d2, size_t(Qs) * k * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&d_sum, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return hip_error(e, "kd_autotune: setup");
    }
    float best = INFINITY;
    kd_opts bo = cands.front();
    uint64_t ref = 0;
    bool have_ref = false;
    for (const kd_opts& o : cands) {
        kd_status s = knn_entry(t, sample_q, Qs, k, maxRadius, idx, d2, nullptr, &o, stream, "kd_autotune");
        if (s != KD_OK) {
            cleanup();
            return s;
        }
        // every candidate must write the same results
        unsigned long long h = 0;
        e = hipMemsetAsync(d_sum, 0, sizeof(h), st);
        if (e == hipSuccess) e = launch_output_checksum(idx, d2, Qs * k, 0, d_sum, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&h, d_sum, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            cleanup();
            return hip_error(e, "kd_autotune: checksum");
        }
        if (have_ref && h != ref) {
            cleanup();
            return set_error(KD_EHIP, "kd_autotune: launch options changed the results");
        }
        ref = h;
        have_ref = true;
        float ms = 0;
        const int reps = 3;
        e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess && s == KD_OK; ++r)
            s = knn_entry(t, sample_q, Qs, k, maxRadius, idx, d2, nullptr, &o, stream, "kd_autotune");
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (s != KD_OK || e != hipSuccess) {
            cleanup();
            return s != KD_OK ? s : hip_error(e, "kd_autotune: timing");
        }
        ms /= reps;
        if (ms < best) {
            best = ms;
            bo = o;
        }
    }
    cleanup();
    set_tuned(t, K, bo);
    if (best_out) *best_out = bo;
    if (best_ms) *best_ms = best;
    return KD_OK;
}

kd_status kd_tree_get_tuned(kd_tree t, int k, kd_opts* out) {
    if (!t || !out) return set_error(KD_EINVAL, "kd_tree_get_tuned: NULL argument");
    if (k < 1 || k > KD_MAX_K) return set_error(KD_EINVAL, "kd_tree_get_tuned: k out of range [1, 64]");
    if (!tuned_opts(t, k_template(k), out)) return set_error(KD_EINVAL, "kd_tree_get_tuned: not tuned for this k");
    return KD_OK;
}

kd_status kd_tree_set_tuned(kd_tree t, int k, const kd_opts* o) {
    if (!t || !o) return set_error(KD_EINVAL, "kd_tree_set_tuned: NULL argument");
    if (k < 1 || k > KD_MAX_K) return set_error(KD_EINVAL, "kd_tree_set_tuned: k out of range [1, 64]");
    QueryPlan p;
    kd_status s = resolve_plan_public(t, k, INFINITY, o, p);
    if (s != KD_OK) return s;
    set_tuned(t, k_template(k), *o);
    return KD_OK;
}

}  // extern "C"
