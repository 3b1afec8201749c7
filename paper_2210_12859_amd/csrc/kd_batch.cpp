// kd_batch.cpp -- many independent trees and query sets in one call.
//
// Jobs are grouped by (dimension, compiled list size K).  For each class the
// jobs' queries form one slot space; the class pipeline is a Morton sort of
// the whole space (job index in the top bits, so every job stays contiguous
// and is sorted along its own tree's Z-order curve), a gather into 32-byte
// query records, and ONE persistent traversal launch whose lanes each carry
// their own tree.  kd_batch_create captures the pipelines of all classes into
// a hipGraph once; kd_batch_run replays it.
#include <hip/hip_runtime.h>

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
        void* ws = nullptr;          // sort scratch, records, cursors
    };
    std::vector<Class> classes;
    std::vector<std::pair<int32_t*, float*>> empty_out;  // jobs over empty trees
    std::vector<int64_t> empty_n;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t total_queries = 0;
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

void free_batch(kd_batch b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& c : b->classes) {
        if (c.d_jobs) (void)hipFree(c.d_jobs);
        if (c.ws) (void)hipFree(c.ws);
    }
    delete b;
}

}  // namespace

}  // namespace kd

using namespace kd;

extern "C" {

kd_status kd_batch_create(const kd_job* jobs, int n_jobs, const kd_opts* opts, kd_stream stream, kd_batch* out) {
    if (!out) return set_error(KD_EINVAL, "kd_batch_create: out is NULL");
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return set_error(KD_EINVAL, "kd_batch_create: bad job list");
    // validate every job before allocating anything
    for (int i = 0; i < n_jobs; ++i) {
        const kd_job& J = jobs[i];
        const std::string f = "kd_batch_create: job " + std::to_string(i);
        if (!J.tree) return set_error(KD_EINVAL, f + ": tree is NULL");
        if (J.Q < 0 || J.Q >= (int64_t(1) << 31)) return set_error(KD_EINVAL, f + ": Q out of range");
        if (J.k < 1 || J.k > KD_MAX_K) return set_error(KD_EINVAL, f + ": k out of range [1, 64]");
        if (std::isnan(J.maxRadius) || J.maxRadius < 0.0f) return set_error(KD_EINVAL, f + ": bad maxRadius");
        if (J.Q > 0 && (!J.queries || !J.out_idx)) return set_error(KD_EINVAL, f + ": NULL pointer");
    }
    QueryPlan plan;
    kd_status s = KD_OK;
    if (n_jobs > 0) {
        s = resolve_plan_public(jobs[0].tree, 1, INFINITY, opts, plan);
        if (s != KD_OK) return s;
    }
    std::unique_ptr<kd_batch_s, void (*)(kd_batch)> b(new kd_batch_s, free_batch);
    int device = 0;
    KD_HIP(hipGetDevice(&device));

    // group by (dim, K); host job tables with class slot bases
    std::map<std::pair<int, int>, std::vector<BatchJob>> groups;
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
        auto& g = groups[{J.tree->dim, K}];
        BatchJob bj{};
        bj.nodes = J.tree->d_nodes;
        // subtree boxes unless the paper's rule alone is asked for
        bj.boxes = plan.prune == 1 ? nullptr : static_cast<const float*>(J.tree->d_boxes);
        bj.box_below = box_id_limit(J.tree->N);
        bj.queries = J.queries;
        bj.out_idx = J.out_idx;
        bj.out_d2 = J.out_d2;
        const int D = J.tree->dim;
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
        uint64_t base = g.empty() ? 0 : uint64_t(g.back().slot_base) + g.back().Q;
        if (base + uint64_t(J.Q) >= (uint64_t(1) << 31))
            return set_error(KD_EINVAL, "kd_batch_create: more than 2^31 queries in one (dim, k) class");
        bj.slot_base = uint32_t(base);
        bj.Q = uint32_t(J.Q);
        bj.vec_store = 0;
        g.push_back(bj);
    }
    for (auto& kv : groups) {
        kd_batch_s::Class c;
        c.dim = kv.first.first;
        c.K = kv.first.second;
        c.njobs = int(kv.second.size());
        c.n = kv.second.back().slot_base + kv.second.back().Q;
        KD_HIP(hipMalloc(&c.d_jobs, kv.second.size() * sizeof(BatchJob)));
        b->classes.push_back(c);  // owned (freed on error) from here on
        KD_HIP(hipMemcpy(b->classes.back().d_jobs, kv.second.data(), kv.second.size() * sizeof(BatchJob),
                         hipMemcpyHostToDevice));
        const size_t sort_b = (batch_sort_scratch_bytes(c.n) + 255) & ~size_t(255);
        const size_t rec_b = (size_t(c.n) * batch_rec_bytes() + 255) & ~size_t(255);
        KD_HIP(hipMalloc(&b->classes.back().ws, sort_b + rec_b + batch_cursor_bytes()));
    }

    // capture the whole batch as one graph (on a private stream when the
    // caller passes the default stream, which cannot be captured)
    hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
    hipStream_t own = nullptr;
    if (!cs) {
        KD_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        cs = own;
    }
    auto fail = [&](kd_status st) {
        if (own) (void)hipStreamDestroy(own);
        return st;
    };
    // One graph branch per (dim, K) class: the classes are independent, so
    // their persistent launches overlap and the long traversals that end one
    // class run beside the next class's work.  Branch streams use the default
    // priority; they fork from and join back into the capture stream.
    std::vector<hipStream_t> side(b->classes.size(), nullptr);
    std::vector<hipEvent_t> done(b->classes.size(), nullptr);
    hipEvent_t fork = nullptr;
    auto release = [&]() {
        for (hipStream_t x : side)
            if (x) (void)hipStreamDestroy(x);
        for (hipEvent_t x : done)
            if (x) (void)hipEventDestroy(x);
        if (fork) (void)hipEventDestroy(fork);
    };
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    for (size_t i = 0; i < side.size() && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release();
        return fail(hip_error(e, "kd_batch_create: branch streams"));
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release();
        return fail(hip_error(e, "kd_batch_create: begin capture"));
    }
    for (size_t i = 0; i < b->empty_out.size(); ++i) {
        const int64_t n = b->empty_n[i];
        hipLaunchKernelGGL(batch_fill_empty, dim3(unsigned((n + 255) / 256)), dim3(256), 0, cs,
                           b->empty_out[i].first, b->empty_out[i].second, n);
    }
    e = hipEventRecord(fork, cs);
    for (size_t i = 0; i < b->classes.size() && s == KD_OK && e == hipSuccess; ++i) {
        auto& c = b->classes[i];
        hipStream_t bs = side[i];
        e = hipStreamWaitEvent(bs, fork, 0);
        if (e != hipSuccess) break;
        char* ws = static_cast<char*>(c.ws);
        const size_t sort_b = (batch_sort_scratch_bytes(c.n) + 255) & ~size_t(255);
        const size_t rec_b = (size_t(c.n) * batch_rec_bytes() + 255) & ~size_t(255);
        const uint32_t* perm = nullptr;
        s = batch_sort(c.d_jobs, c.njobs, c.dim, c.n, plan.sort_bits, ws, bs, &perm);
        if (s != KD_OK) break;
        QueryPlan cp = plan;
        cp.K = c.K;
        s = run_batch_class(c.d_jobs, c.njobs, c.dim, c.K, c.n, perm, ws + sort_b,
                            reinterpret_cast<uint32_t*>(ws + sort_b + rec_b), cp, device, bs);
        if (s != KD_OK) break;
        e = hipEventRecord(done[i], bs);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, done[i], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    release();
    if (s == KD_OK && e != hipSuccess) s = hip_error(e, "kd_batch_create: branch capture");
    e = ec;
    if (s != KD_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(s);
    }
    if (e != hipSuccess) return fail(hip_error(e, "kd_batch_create: end capture"));
    b->graph = graph;
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(hip_error(e, "kd_batch_create: instantiate"));
    if (own) (void)hipStreamDestroy(own);
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

kd_status kd_knn_batched(const kd_job* jobs, int n_jobs, const kd_opts* opts, kd_stream stream) {
    kd_batch b = nullptr;
    kd_status s = kd_batch_create(jobs, n_jobs, opts, stream, &b);
    if (s != KD_OK) return s;
    s = kd_batch_run(b, stream);
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    kd_batch_free(b);
    if (s != KD_OK) return s;
    if (e != hipSuccess) return hip_error(e, "kd_knn_batched: synchronize");
    return KD_OK;
}

}  // extern "C"
