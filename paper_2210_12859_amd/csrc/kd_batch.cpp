// kd_batch.cpp -- many independent trees and query sets in one call.
//
// Jobs are grouped by (dimension, compiled list size K).  For each class the
// jobs' queries form one slot space; the class pipeline is a Morton sort of
// the whole space (job index in the top bits, so every job stays contiguous
// and is sorted along its own tree's Z-order curve), a gather into 32-byte
// query records, the initial radii of the jobs that have a radius model (3-D),
// ONE persistent traversal launch whose lanes each carry their own tree, and
// the cooperative kernel for the queries that ran over the trip budget.
// kd_batch_create captures the pipelines of all classes into a hipGraph once;
// kd_batch_run replays it; kd_batch_autotune times launch options per class
// and captures the graph again with the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "kd_internal.h"

struct kd_batch_s {
    struct Class {
        int dim = 0, K = 0;
        uint32_t n = 0;
        int njobs = 0;
        kd::BatchJob* d_jobs = nullptr;
        std::vector<kd::BatchJob> jobs;  // host copy (output pointers for the autotuner's checksum)
        void* ws = nullptr;              // sort scratch | records | counters | hand-off rows | initial radii
        kd::MlpJob* d_mlp = nullptr;     // radius-model table of the class's jobs with a model
        int n_mlp = 0;
        uint32_t mlp_tiles = 0;
        kd::QueryPlan plan;
        float est_ms = 0.0f;             // expected pipeline time: measured by the autotuner, else estimated
    };
    std::vector<Class> classes;
    std::vector<std::pair<int32_t*, float*>> empty_out;  // jobs over empty trees
    std::vector<int64_t> empty_n;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t total_queries = 0;
    int device = 0;
};

namespace kd {

namespace {

__global__ void batch_fill_empty(int32_t* idx, float* d2, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        idx[i] = -1;
        if (d2) d2[i] = __builtin_inff();
    }
}

// Order-independent, position-sensitive 64-bit checksum of one job's outputs,
// folded into *h (the autotuner checks that every candidate gives the same).
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

__global__ void output_checksum(const int32_t* idx, const float* d2, int64_t n, uint64_t salt,
                                unsigned long long* h) {
    uint64_t acc = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const uint64_t v = uint64_t(uint32_t(idx[i])) | (d2 ? uint64_t(__float_as_uint(d2[i])) << 32 : 0);
        acc ^= mix64(v ^ mix64(uint64_t(i) ^ salt));
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        acc ^= uint64_t(uint32_t(__shfl_xor(uint32_t(acc), m))) |
               (uint64_t(uint32_t(__shfl_xor(uint32_t(acc >> 32), m))) << 32);
    if ((threadIdx.x & 63) == 0 && acc) atomicXor(h, (unsigned long long)acc);
}

}  // namespace

hipError_t launch_output_checksum(const int32_t* idx, const float* d2, int64_t n, uint64_t salt,
                                  unsigned long long* h, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = unsigned(std::min<int64_t>((n + 255) / 256, 1024));
    hipLaunchKernelGGL(output_checksum, dim3(blocks), dim3(256), 0, st, idx, d2, n, salt, h);
    return hipGetLastError();
}

namespace {

void free_batch(kd_batch b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& c : b->classes) {
        if (c.d_jobs) (void)hipFree(c.d_jobs);
        if (c.ws) (void)hipFree(c.ws);
        if (c.d_mlp) (void)hipFree(c.d_mlp);
    }
    delete b;
}

struct ClassLayout {
    size_t sort_b, rec_b, cur_b, heavy_b, w0_b;
};

ClassLayout class_layout(const kd_batch_s::Class& c, int device) {
    ClassLayout L;
    L.sort_b = (batch_sort_scratch_bytes(c.n) + 255) & ~size_t(255);
    L.rec_b = (size_t(c.n) * batch_rec_bytes() + 255) & ~size_t(255);
    L.cur_b = (batch_cursor_bytes() + 255) & ~size_t(255);
    L.heavy_b = (size_t(batch_heavy_cap(device)) * 8 + 255) & ~size_t(255);
    L.w0_b = c.n_mlp ? (size_t(c.n) * 4 + 255) & ~size_t(255) : 0;
    return L;
}

#ifndef KD_BATCH_BRANCHES
#define KD_BATCH_BRANCHES 3
#endif

// Rough time of a group's pipeline, from the measured single-tree cost per
// query on 1M-point trees (fcp 0.25 ms, k = 8 0.67 ms, k = 64 6.4 ms per 1M
// 3-D queries; 4-D about 1.7x, 2-D 0.7x).  Only the order in which the groups
// are captured depends on it.
float class_cost_estimate(int dim, int K, uint32_t n) {
    float kf = 1.0f;
    switch (K) {
        case 1: kf = 0.37f; break;
        case 2: kf = 0.5f; break;
        case 4: kf = 0.65f; break;
        case 8: kf = 1.0f; break;
        case 16: kf = 1.9f; break;
        case 32: kf = 3.8f; break;
        default: kf = 9.5f; break;
    }
    const float df = dim == 2 ? 0.7f : (dim == 3 ? 1.0f : 1.7f);
    return float(n) * 0.67e-6f * kf * df;
}

// The whole pipeline of one class on stream st.
kd_status enqueue_class(const kd_batch_s::Class& c, int device, hipStream_t st) {
    const ClassLayout L = class_layout(c, device);
    char* ws = static_cast<char*>(c.ws);
    const uint32_t* perm = nullptr;
    kd_status s = batch_sort(c.d_jobs, c.njobs, c.dim, c.n, c.plan.sort_bits, ws, st, &perm);
    if (s != KD_OK) return s;
    char* recs = ws + L.sort_b;
    uint32_t* counters = reinterpret_cast<uint32_t*>(recs + L.rec_b);
    int32_t* heavy = reinterpret_cast<int32_t*>(recs + L.rec_b + L.cur_b);
    BatchLearned bl{c.d_mlp, c.n_mlp, c.mlp_tiles,
                    c.n_mlp ? reinterpret_cast<float*>(recs + L.rec_b + L.cur_b + L.heavy_b) : nullptr};
    return run_batch_class(c.d_jobs, c.njobs, c.dim, c.K, c.n, perm, recs, counters, c.plan, device, st,
                           c.n_mlp ? &bl : nullptr, heavy);
}

// Captures every class into one graph: one graph branch per (dim, K) class
// (the classes are independent, so their persistent launches overlap and the
// long traversals that end one class run beside the next class's work).
// Branch streams use the default priority; they fork from and join back into
// the capture stream, which is a private one when the caller passes the
// default stream (that stream cannot be captured).
kd_status capture_batch(kd_batch b, hipStream_t cs_in) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    hipStream_t cs = cs_in;
    hipStream_t own = nullptr;
    if (!cs) {
        KD_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        cs = own;
    }
    // The groups run on a few graph branches, each a chain of groups: longest
    // group first onto the least loaded branch (by expected time).  The
    // branches share the device's hardware queues, so more branches than
    // queues would only serialize behind each other in an order the runtime
    // picks.
    const size_t nb = std::min<size_t>(b->classes.size(), KD_BATCH_BRANCHES);
    std::vector<size_t> order(b->classes.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return b->classes[x].est_ms > b->classes[y].est_ms; });
    std::vector<std::vector<size_t>> chain(nb);
    std::vector<float> load(nb, 0.0f);
    for (size_t i : order) {
        const size_t j = size_t(std::min_element(load.begin(), load.end()) - load.begin());
        chain[j].push_back(i);
        load[j] += b->classes[i].est_ms;
    }
    std::vector<hipStream_t> side(nb, nullptr);
    std::vector<hipEvent_t> done(nb, nullptr);
    hipEvent_t fork = nullptr;
    auto release = [&]() {
        for (hipStream_t x : side)
            if (x) (void)hipStreamDestroy(x);
        for (hipEvent_t x : done)
            if (x) (void)hipEventDestroy(x);
        if (fork) (void)hipEventDestroy(fork);
        if (own) (void)hipStreamDestroy(own);
    };
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    for (size_t i = 0; i < side.size() && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release();
        return hip_error(e, "kd_batch: branch streams");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release();
        return hip_error(e, "kd_batch: begin capture");
    }
    for (size_t i = 0; i < b->empty_out.size(); ++i) {
        const int64_t n = b->empty_n[i];
        hipLaunchKernelGGL(batch_fill_empty, dim3(unsigned((n + 255) / 256)), dim3(256), 0, cs,
                           b->empty_out[i].first, b->empty_out[i].second, n);
    }
    kd_status s = KD_OK;
    e = hipEventRecord(fork, cs);
    for (size_t i = 0; i < nb && s == KD_OK && e == hipSuccess; ++i) {
        e = hipStreamWaitEvent(side[i], fork, 0);
        if (e != hipSuccess) break;
        for (size_t c : chain[i]) {
            s = enqueue_class(b->classes[c], b->device, side[i]);
            if (s != KD_OK) break;
        }
        if (s != KD_OK) break;
        e = hipEventRecord(done[i], side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, done[i], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    release();
    if (s == KD_OK && e != hipSuccess) s = hip_error(e, "kd_batch: branch capture");
    if (s == KD_OK && ec != hipSuccess) s = hip_error(ec, "kd_batch: end capture");
    if (s != KD_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    b->graph = graph;
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_error(e, "kd_batch: instantiate");
    return KD_OK;
}

}  // namespace

}  // namespace kd

using namespace kd;

extern "C" {

kd_status kd_batch_create(const kd_job* jobs, int n_jobs, kd_model model, const kd_opts* opts, kd_stream stream,
                          kd_batch* out) {
    if (!out) return set_error(KD_EINVAL, "kd_batch_create: out is NULL");
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return set_error(KD_EINVAL, "kd_batch_create: bad job list");
    // validate every job before allocating anything
    for (int i = 0; i < n_jobs; ++i) {
        const kd_job& J = jobs[i];
        const std::string f = "kd_batch_create: job " + std::to_string(i);
        if (!J.tree) return set_error(KD_EINVAL, f + ": tree is NULL");
        if (J.tree->split != KD_SPLIT_LEVEL)
            return set_error(KD_EUNSUPPORTED, f + ": trees with stored split dimensions are not batched");
        if (J.Q < 0 || J.Q >= (int64_t(1) << 31)) return set_error(KD_EINVAL, f + ": Q out of range");
        if (J.k < 1 || J.k > KD_MAX_K) return set_error(KD_EINVAL, f + ": k out of range [1, 64]");
        if (std::isnan(J.maxRadius) || J.maxRadius < 0.0f) return set_error(KD_EINVAL, f + ": bad maxRadius");
        if (J.Q > 0 && (!J.queries || !J.out_idx)) return set_error(KD_EINVAL, f + ": NULL pointer");
    }
    // options shared by every class; the list size of each class sets its
    // default persistent grid
    QueryPlan base;
    kd_status s = resolve_plan_public(nullptr, 1, INFINITY, opts, base);
    if (s != KD_OK) return s;
    std::unique_ptr<kd_batch_s, void (*)(kd_batch)> b(new kd_batch_s, free_batch);
    KD_HIP(hipGetDevice(&b->device));

    // group by (dim, K); host job tables with class slot bases, and the
    // radius-model table of the 3-D jobs with a model
    std::map<std::pair<int, int>, std::vector<BatchJob>> groups;
    std::map<std::pair<int, int>, std::vector<MlpJob>> mlp;
    for (int i = 0; i < n_jobs; ++i) {
        const kd_job& J = jobs[i];
        b->total_queries += J.Q;
        if (J.Q == 0) continue;
        if (J.tree->N == 0) {
            b->empty_out.emplace_back(J.out_idx, J.out_d2);
            b->empty_n.push_back(J.Q * J.k);
            continue;
        }
        const int K = k_template(J.k);
        const int D = J.tree->dim;
        auto& g = groups[{D, K}];
        BatchJob bj{};
        bj.nodes = J.tree->d_nodes;
        // subtree boxes unless the paper's rule alone is asked for
        bj.boxes = base.prune == 1 ? nullptr : static_cast<const float*>(J.tree->d_boxes);
        bj.box_below = box_id_limit(J.tree->N);
        bj.queries = J.queries;
        bj.out_idx = J.out_idx;
        bj.out_d2 = J.out_d2;
        const int bits = D == 2 ? 16 : (D == 3 ? 10 : 8);
        for (int d = 0; d < 4; ++d) {
            const float ext = J.tree->hi[d] - J.tree->lo[d];
            bj.lo[d] = J.tree->lo[d];
            bj.scale[d] = (d < D && ext > 0.0f) ? float(1u << bits) / ext : 0.0f;
        }
        bj.N = int32_t(J.tree->N);
        bj.k = J.k;
        const float r = J.maxRadius;
        bj.R2 = r * r;
        uint64_t start = g.empty() ? 0 : uint64_t(g.back().slot_base) + g.back().Q;
        if (start + uint64_t(J.Q) >= (uint64_t(1) << 31))
            return set_error(KD_EINVAL, "kd_batch_create: more than 2^31 queries in one (dim, k) class");
        bj.slot_base = uint32_t(start);
        bj.Q = uint32_t(J.Q);
        bj.vec_store = 0;
        const kd_model m = J.model ? J.model : model;
        bj.learned = 0;
        if (m && D == 3) {
            MlpJob mj{};
            s = model_view(m, &mj);
            if (s != KD_OK) return s;
            auto& mt = mlp[{D, K}];
            mj.R2 = bj.R2;
            mj.slot_base = bj.slot_base;
            mj.Q = bj.Q;
            mj.tile_base = mt.empty() ? 0 : mt.back().tile_base + (mt.back().Q + 63) / 64;
            mt.push_back(mj);
            bj.learned = 1;
        }
        g.push_back(bj);
    }
    for (auto& kv : groups) {
        kd_batch_s::Class c;
        c.dim = kv.first.first;
        c.K = kv.first.second;
        c.njobs = int(kv.second.size());
        c.n = kv.second.back().slot_base + kv.second.back().Q;
        c.jobs = kv.second;
        c.plan = base;
        c.plan.K = c.K;
        if (!opts || opts->waves_per_cu == 0) c.plan.waves_per_cu = c.K == 1 ? 32 : 24;
        if (!opts || opts->sort_bits < 0) {
            // the job index takes the top bits of the sort key: keep 16 bits
            // of Morton code below it
            int jb = 0;
            while ((1 << jb) < c.njobs) ++jb;
            c.plan.sort_bits = std::min(32, ((jb + 16 + 7) / 8) * 8);
        }
        c.est_ms = class_cost_estimate(c.dim, c.K, c.n);
        b->classes.push_back(c);  // owned (freed on error) from here on
        kd_batch_s::Class& cc = b->classes.back();
        KD_HIP(hipMalloc(&cc.d_jobs, kv.second.size() * sizeof(BatchJob)));
        KD_HIP(hipMemcpy(cc.d_jobs, kv.second.data(), kv.second.size() * sizeof(BatchJob), hipMemcpyHostToDevice));
        auto it = mlp.find(kv.first);
        if (it != mlp.end()) {
            cc.n_mlp = int(it->second.size());
            cc.mlp_tiles = it->second.back().tile_base + (it->second.back().Q + 63) / 64;
            KD_HIP(hipMalloc(&cc.d_mlp, it->second.size() * sizeof(MlpJob)));
            KD_HIP(hipMemcpy(cc.d_mlp, it->second.data(), it->second.size() * sizeof(MlpJob), hipMemcpyHostToDevice));
        }
        const ClassLayout L = class_layout(cc, b->device);
        KD_HIP(hipMalloc(&cc.ws, L.sort_b + L.rec_b + L.cur_b + L.heavy_b + L.w0_b));
    }
    s = capture_batch(b.get(), reinterpret_cast<hipStream_t>(stream));
    if (s != KD_OK) return s;
    *out = b.release();
    return KD_OK;
}

kd_status kd_batch_run(kd_batch b, kd_stream stream) {
    if (!b) return set_error(KD_EINVAL, "kd_batch_run: batch is NULL");
    KD_HIP(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
    return KD_OK;
}

kd_status kd_batch_free(kd_batch b) {
    free_batch(b);
    return KD_OK;
}

kd_status kd_knn_batched(const kd_job* jobs, int n_jobs, kd_model model, const kd_opts* opts, kd_stream stream) {
    kd_batch b = nullptr;
    kd_status s = kd_batch_create(jobs, n_jobs, model, opts, stream, &b);
    if (s != KD_OK) return s;
    s = kd_batch_run(b, stream);
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    kd_batch_free(b);
    if (s != KD_OK) return s;
    if (e != hipSuccess) return hip_error(e, "kd_knn_batched: synchronize");
    return KD_OK;
}

kd_status kd_batch_autotune(kd_batch b, int reps, kd_stream stream, kd_opts* class_opts, int* n_classes) {
    if (!b) return set_error(KD_EINVAL, "kd_batch_autotune: batch is NULL");
    if (reps < 1) reps = 3;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipStream_t own = nullptr;
    if (!st) {
        KD_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        st = own;
    }
    unsigned long long* d_sum = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (d_sum) (void)hipFree(d_sum);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (own) (void)hipStreamDestroy(own);
    };
    hipError_t e = hipMalloc(&d_sum, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return hip_error(e, "kd_batch_autotune: setup");
    }
    // the checksum of a class's outputs after one run of its pipeline
    auto checksum = [&](const kd_batch_s::Class& c, uint64_t* h) -> kd_status {
        KD_HIP(hipMemsetAsync(d_sum, 0, sizeof(unsigned long long), st));
        for (size_t j = 0; j < c.jobs.size(); ++j) {
            const BatchJob& J = c.jobs[j];
            KD_HIP(launch_output_checksum(J.out_idx, J.out_d2, int64_t(J.Q) * J.k, uint64_t(j) << 40, d_sum, st));
        }
        unsigned long long v = 0;
        KD_HIP(hipMemcpyAsync(&v, d_sum, sizeof(v), hipMemcpyDeviceToHost, st));
        KD_HIP(hipStreamSynchronize(st));
        *h = v;
        return KD_OK;
    };
    kd_status s = KD_OK;
    for (auto& c : b->classes) {
        // candidates: workgroup size x waves per CU x Morton sort bits
        const QueryPlan keep = c.plan;
        QueryPlan best = keep;
        float best_ms = INFINITY;
        uint64_t ref = 0;
        bool have_ref = false;
        for (int block : {256, 512}) {
            if (c.K >= 32 && block > 256) continue;
            for (int wpc : {16, 24, 32}) {
                for (int bits : {16, 24, 32}) {
                    c.plan = keep;
                    c.plan.block = block;
                    c.plan.waves_per_cu = wpc;
                    c.plan.sort_bits = bits;
                    s = enqueue_class(c, b->device, st);  // warm-up, and the outputs to check
                    uint64_t h = 0;
                    if (s == KD_OK) s = checksum(c, &h);
                    if (s == KD_OK && have_ref && h != ref)
                        s = set_error(KD_EHIP, "kd_batch_autotune: launch options changed the results");
                    if (s != KD_OK) break;
                    ref = h;
                    have_ref = true;
                    hipError_t er = hipEventRecord(e0, st);
                    for (int r = 0; r < reps && s == KD_OK && er == hipSuccess; ++r) s = enqueue_class(c, b->device, st);
                    if (er == hipSuccess) er = hipEventRecord(e1, st);
                    if (er == hipSuccess) er = hipEventSynchronize(e1);
                    float ms = 0;
                    if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
                    if (s == KD_OK && er != hipSuccess) s = hip_error(er, "kd_batch_autotune: timing");
                    if (s != KD_OK) break;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = c.plan;
                    }
                }
                if (s != KD_OK) break;
            }
            if (s != KD_OK) break;
        }
        c.plan = s == KD_OK ? best : keep;
        if (s == KD_OK) c.est_ms = best_ms / float(reps);
        if (s != KD_OK) break;
    }
    if (s == KD_OK) s = capture_batch(b, reinterpret_cast<hipStream_t>(stream));
    if (s == KD_OK && n_classes) {
        const int cap = *n_classes;
        *n_classes = int(b->classes.size());
        for (int i = 0; class_opts && i < cap && i < int(b->classes.size()); ++i) {
            const QueryPlan& p = b->classes[i].plan;
            class_opts[i] = kd_opts{p.block, p.lds_levels, p.sort_bits, p.waves_per_cu,
                                    p.heavy_default ? 0 : (p.heavy_trips > 0 ? p.heavy_trips : -1), p.prune};
        }
    }
    cleanup();
    return s;
}

kd_status kd_batch_info(kd_batch b, int* n_classes, int* class_dim, int* class_k, int64_t* class_queries, int cap) {
    if (!b || !n_classes) return set_error(KD_EINVAL, "kd_batch_info: NULL argument");
    *n_classes = int(b->classes.size());
    for (int i = 0; i < cap && i < int(b->classes.size()); ++i) {
        if (class_dim) class_dim[i] = b->classes[i].dim;
        if (class_k) class_k[i] = b->classes[i].K;
        if (class_queries) class_queries[i] = b->classes[i].n;
    }
    return KD_OK;
}

}  // extern "C"
