// kd_api.cpp -- the C ABI of libkdtree: argument validation, error state,
// tree objects, per-stream scratch, and dispatch into the HIP pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "kd_internal.h"

namespace kd {

namespace {
thread_local std::string g_last_error;

std::mutex g_dev_mu;
std::map<int, DeviceInfo> g_dev;

struct ScratchBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_scratch_mu;
std::map<std::pair<int, kd_stream>, ScratchBuf> g_scratch;
std::map<std::pair<int, kd_stream>, ScratchBuf> g_aux_scratch;
}  // namespace

kd_status set_error(kd_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

kd_status hip_error(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? KD_ENOMEM : KD_EHIP;
}

const DeviceInfo& device_info(int device) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev.find(device);
    if (it != g_dev.end()) return it->second;
    DeviceInfo di;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) == hipSuccess) {
        di.cus = p.multiProcessorCount;
        di.lds_bytes = int(p.sharedMemPerBlock);
    }
    return g_dev.emplace(device, di).first->second;
}

namespace {
struct TimedLaunch {
    std::string kernel;
    hipEvent_t a, b;
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<TimedLaunch> g_timed;
}  // namespace

bool timing_enabled() {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    return g_timing_on;
}

kd_status timing_begin(hipStream_t st, hipEvent_t* ev) {
    *ev = nullptr;
    if (!timing_enabled()) return KD_OK;
    KD_HIP(hipEventCreate(ev));
    KD_HIP(hipEventRecord(*ev, st));
    return KD_OK;
}

kd_status timing_end(hipStream_t st, hipEvent_t ev0, const char* kernel) {
    if (!ev0) return KD_OK;
    hipEvent_t ev1;
    KD_HIP(hipEventCreate(&ev1));
    KD_HIP(hipEventRecord(ev1, st));
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timed.push_back({kernel, ev0, ev1});
    return KD_OK;
}

namespace {
kd_status grow_scratch(std::map<std::pair<int, kd_stream>, ScratchBuf>& m, kd_stream stream, size_t bytes,
                       void** out) {
    int dev = 0;
    KD_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchBuf& b = m[{dev, stream}];
    if (b.bytes < bytes) {
        if (b.ptr) {
            // the stream may still use the old buffer
            KD_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
            KD_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t sz = bytes < (1u << 20) ? (1u << 20) : bytes + bytes / 4;
        KD_HIP(hipMalloc(&b.ptr, sz));
        b.bytes = sz;
    }
    *out = b.ptr;
    return KD_OK;
}
}  // namespace

kd_status scratch(kd_stream stream, size_t bytes, void** out) { return grow_scratch(g_scratch, stream, bytes, out); }

kd_status aux_scratch(kd_stream stream, size_t bytes, void** out) {
    return grow_scratch(g_aux_scratch, stream, bytes, out);
}

namespace {

// Record of node id i (1-based, id = level-order position + 1) at array index
// i; index 0 and index N + 1 are zero padding, so the two children of any node
// (ids 2c, 2c + 1) sit in one aligned pair and a pair read never leaves the
// allocation.
template <int D>
void pack_records(const float* pts, const int32_t* order, int64_t N, std::vector<unsigned char>& out) {
    out.assign(node_buffer_bytes(D, N), 0);
    TreeRec<D>* r = reinterpret_cast<TreeRec<D>*>(out.data());
    int32_t* ids = reinterpret_cast<int32_t*>(r + (N + 2));  // used when the record holds no index
    constexpr int A0 = D + (rec_has_idx(D) ? 1 : 0);          // first ancestor word
    for (int64_t pos = 0; pos < N; ++pos) {
        TreeRec<D>& rec = r[pos + 1];
        const int32_t i = order[pos];
        for (int j = 0; j < D; ++j) std::memcpy(&rec.w[j], &pts[int64_t(i) * D + j], 4);
        if (rec_has_idx(D)) rec.w[D] = uint32_t(i);
        else ids[pos + 1] = i;
        // ancestors by 1-based id: a = (pos+1) >> m, level floor(log2 a)
        int64_t a = (pos + 1) >> 1;
        for (int m = 0; m < rec_ancestors(D); ++m, a >>= 1) {
            if (a < 1) break;
            const int lvl = 63 - __builtin_clzll((unsigned long long)a);
            std::memcpy(&rec.w[A0 + m], &pts[int64_t(order[a - 1]) * D + (lvl % D)], 4);
        }
    }
}

// Bounding box of the points of every subtree, children before parents:
// node id i (1-based) covers its own point and the boxes of ids 2i, 2i + 1.
void pack_boxes(const float* pts, const int32_t* order, int64_t N, int D, std::vector<float>& out) {
    const int BW = box_words(D), H = BW / 2;
    out.assign(size_t(N + 2) * BW, 0.0f);
    for (int64_t id = N; id >= 1; --id) {
        float* b = &out[size_t(id) * BW];
        const float* p = &pts[int64_t(order[id - 1]) * D];
        for (int j = 0; j < D; ++j) b[j] = b[H + j] = p[j];
        for (int64_t c = 2 * id; c <= 2 * id + 1 && c <= N; ++c) {
            const float* cb = &out[size_t(c) * BW];
            for (int j = 0; j < D; ++j) {
                b[j] = std::min(b[j], cb[j]);
                b[H + j] = std::max(b[H + j], cb[H + j]);
            }
        }
    }
}

kd_status build_from_host(const float* hp, int64_t N, int dim, kd_tree* out) {
    if (!out) return set_error(KD_EINVAL, "kd_build: out is NULL");
    if (N < 0 || N > KD_MAX_POINTS) return set_error(KD_EINVAL, "kd_build: N out of range [0, 2^30 - 1]");
    if (dim < 2 || dim > 4) return set_error(KD_EINVAL, "kd_build: dim must be 2, 3 or 4");
    if (N > 0 && !hp) return set_error(KD_EINVAL, "kd_build: points is NULL");
    for (int64_t i = 0; i < N * dim; ++i)
        if (!std::isfinite(hp[i])) return set_error(KD_EINVAL, "kd_build: points contain NaN or inf");
    std::unique_ptr<kd_tree_s> t(new (std::nothrow) kd_tree_s);
    if (!t) return set_error(KD_ENOMEM, "kd_build: host allocation");
    t->N = N;
    t->dim = dim;
    KD_HIP(hipGetDevice(&t->device));
    for (int j = 0; j < 4; ++j) { t->lo[j] = 0; t->hi[j] = 0; }
    if (N > 0) {
        for (int j = 0; j < dim; ++j) { t->lo[j] = hp[j]; t->hi[j] = hp[j]; }
        for (int64_t i = 1; i < N; ++i)
            for (int j = 0; j < dim; ++j) {
                float v = hp[i * dim + j];
                if (v < t->lo[j]) t->lo[j] = v;
                if (v > t->hi[j]) t->hi[j] = v;
            }
    }
    try {
        t->order.resize(size_t(N));
    } catch (...) {
        return set_error(KD_ENOMEM, "kd_build: host allocation");
    }
    build_level_order(hp, N, dim, t->order.data(), 0);
    if (N > 0) {
        std::vector<unsigned char> recs;
        if (dim == 2) pack_records<2>(hp, t->order.data(), N, recs);
        else if (dim == 3) pack_records<3>(hp, t->order.data(), N, recs);
        else pack_records<4>(hp, t->order.data(), N, recs);
        KD_HIP(hipMalloc(&t->d_nodes, recs.size()));
        hipError_t e = hipMemcpy(t->d_nodes, recs.data(), recs.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(t->d_nodes);
            return hip_error(e, "kd_build: upload");
        }
        std::vector<unsigned char>().swap(recs);
        std::vector<float> boxes;
        try {
            pack_boxes(hp, t->order.data(), N, dim, boxes);
        } catch (...) {
            (void)hipFree(t->d_nodes);
            return set_error(KD_ENOMEM, "kd_build: host allocation");
        }
        e = hipMalloc(&t->d_boxes, boxes.size() * 4);
        if (e == hipSuccess) e = hipMemcpy(t->d_boxes, boxes.data(), boxes.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(t->d_nodes);
            if (t->d_boxes) (void)hipFree(t->d_boxes);
            return hip_error(e, "kd_build: upload");
        }
    }
    *out = t.release();
    return KD_OK;
}

kd_status check_query_args(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius,
                           const int32_t* out_idx, const char* fn) {
    std::string f(fn);
    if (Q < 0 || Q >= (int64_t(1) << 31)) return set_error(KD_EINVAL, f + ": Q out of range [0, 2^31)");
    if (k < 1 || k > KD_MAX_K) return set_error(KD_EINVAL, f + ": k out of range [1, 64]");
    if (std::isnan(maxRadius) || maxRadius < 0.0f) return set_error(KD_EINVAL, f + ": maxRadius must be >= 0 or +inf");
    if (!t) return set_error(KD_EINVAL, f + ": tree is NULL");
    if (Q > 0 && !queries) return set_error(KD_EINVAL, f + ": queries is NULL");
    if (Q > 0 && !out_idx) return set_error(KD_EINVAL, f + ": out_idx is NULL");
    return KD_OK;
}

__global__ void fill_empty(int32_t* idx, float* d2, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        idx[i] = -1;
        if (d2) d2[i] = __builtin_inff();
    }
}

__global__ void fill_zero_u32(uint32_t* p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

kd_status resolve_plan(kd_tree t, int k, float maxRadius, const kd_opts* o, QueryPlan& p) {
    p.k = k;
    p.K = k_template(k);
    float r = maxRadius;
    p.R2 = r * r;  // binary32 product; +inf stays +inf
    kd_opts use{0, -1, -1, 0, 0, 0};
    kd_opts tuned;
    if (o) use = *o;
    else if (t && tuned_opts(t, p.K, &tuned)) {
        use = tuned;
        // a tuned box rule is the default rule, which still gives the
        // paper's count when visited is requested
        if (use.prune == 2) use.prune = 0;
    }
    if (use.block == 0) use.block = 256;
    if (use.lds_levels < 0) use.lds_levels = 0;
    if (use.sort_bits < 0) use.sort_bits = 16;
    if (use.waves_per_cu == 0) use.waves_per_cu = p.K == 1 ? 32 : 24;  // measured best on 1M uniform
    p.heavy_default = use.heavy_trips == 0;
    if (use.heavy_trips == 0) use.heavy_trips = KD_DEFAULT_HEAVY_TRIPS;
    if (use.heavy_trips < -1) return set_error(KD_EINVAL, "opts.heavy_trips must be -1, 0 or positive");
    if (use.block != 64 && use.block != 128 && use.block != 256 && use.block != 512 && use.block != 1024)
        return set_error(KD_EINVAL, "opts.block must be 64, 128, 256, 512 or 1024");
    if (use.lds_levels > 12) return set_error(KD_EINVAL, "opts.lds_levels must be <= 12");
    if (t && t->d_dims && use.lds_levels > 0)
        return set_error(KD_EINVAL, "opts.lds_levels must be 0 for trees with stored split dimensions");
    if (t && use.lds_levels > 0 && (size_t(1) << use.lds_levels) * 4 * size_t(rec_words(t->dim)) > 65536)
        return set_error(KD_EINVAL, "opts.lds_levels: the staged levels exceed 64 KB of LDS (dim 4: at most 11)");
    if (use.sort_bits > 32) return set_error(KD_EINVAL, "opts.sort_bits must be in 0..32 or -1");
    use.sort_bits = ((use.sort_bits + 7) / 8) * 8;  // the radix sort takes whole bytes
    if (use.waves_per_cu < 1 || use.waves_per_cu > 32) return set_error(KD_EINVAL, "opts.waves_per_cu must be in 1..32");
    if (use.prune < 0 || use.prune > 2) return set_error(KD_EINVAL, "opts.prune must be 0, 1 or 2");
    p.block = use.block;
    p.lds_levels = use.lds_levels;
    p.sort_bits = use.sort_bits;
    p.waves_per_cu = use.waves_per_cu;
    p.heavy_trips = use.heavy_trips > 0 ? use.heavy_trips : 0;
    p.prune = use.prune;
    return KD_OK;
}

}  // namespace

kd_status resolve_plan_public(kd_tree t, int k, float maxRadius, const kd_opts* o, QueryPlan& p) {
    return resolve_plan(t, k, maxRadius, o, p);
}

kd_status check_query_args_public(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius,
                                  const int32_t* out_idx, const char* fn) {
    return check_query_args(t, queries, Q, k, maxRadius, out_idx, fn);
}

kd_status knn_entry(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius, int32_t* out_idx,
                    float* out_d2, uint32_t* visited, const kd_opts* opts, kd_stream stream, const char* fn,
                    const FixedScratch* fixed) {
    kd_status s = check_query_args(t, queries, Q, k, maxRadius, out_idx, fn);
    if (s != KD_OK) return s;
    QueryPlan plan;
    s = resolve_plan(t, k, maxRadius, opts, plan);
    if (s != KD_OK) return s;
    if (Q == 0) return KD_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (t->N == 0) {
        // empty tree: every slot is empty; the traversal is never entered
        int64_t n = Q * k;
        hipLaunchKernelGGL(fill_empty, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, out_idx, out_d2, n);
        KD_HIP(hipGetLastError());
        if (visited) {
            hipLaunchKernelGGL(fill_zero_u32, dim3(unsigned((Q + 255) / 256)), dim3(256), 0, st, visited, Q);
            KD_HIP(hipGetLastError());
        }
        return KD_OK;
    }
    return run_knn(t, queries, Q, plan, out_idx, out_d2, visited, stream, nullptr, nullptr, fixed);
}

}  // namespace kd

using namespace kd;

extern "C" {

kd_status kd_build_host(const float* host_points, int64_t N, int dim, kd_tree* out) {
    try {
        return build_from_host(host_points, N, dim, out);
    } catch (const std::exception& e) {
        return set_error(KD_ENOMEM, std::string("kd_build: ") + e.what());
    }
}

kd_status kd_build(const float* points, int64_t N, int dim, kd_stream stream, kd_tree* out) {
    return kd_build_ex(points, N, dim, KD_SPLIT_LEVEL, stream, out);
}

kd_status kd_build_ex(const float* points, int64_t N, int dim, int split, kd_stream stream, kd_tree* out) {
    if (!out) return set_error(KD_EINVAL, "kd_build: out is NULL");
    if (split != KD_SPLIT_LEVEL && split != KD_SPLIT_WIDEST)
        return set_error(KD_EINVAL, "kd_build: split must be KD_SPLIT_LEVEL or KD_SPLIT_WIDEST");
    if (N < 0 || N > KD_MAX_POINTS) return set_error(KD_EINVAL, "kd_build: N out of range [0, 2^30 - 1]");
    if (dim < 2 || dim > 4) return set_error(KD_EINVAL, "kd_build: dim must be 2, 3 or 4");
    if (N > 0 && !points) return set_error(KD_EINVAL, "kd_build: points is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    bool finite = true;
    kd_status s = check_points_finite(points, N, dim, st, &finite);
    if (s != KD_OK) return s;
    if (!finite) return set_error(KD_EINVAL, "kd_build: points contain NaN or inf");
    std::unique_ptr<kd_tree_s> t(new (std::nothrow) kd_tree_s);
    if (!t) return set_error(KD_ENOMEM, "kd_build: host allocation");
    t->N = N;
    t->dim = dim;
    t->split = split;
    KD_HIP(hipGetDevice(&t->device));
    for (int j = 0; j < 4; ++j) t->lo[j] = t->hi[j] = 0.0f;
    if (N == 0) {
        *out = t.release();
        return KD_OK;
    }
    try {
        t->order.resize(size_t(N));
    } catch (...) {
        return set_error(KD_ENOMEM, "kd_build: host allocation");
    }
    // level order, node records and subtree boxes on the device
    int32_t* d_order = nullptr;
    KD_HIP(hipMalloc(&d_order, size_t(N) * 4));
    struct FreeOrder {
        int32_t* p;
        ~FreeOrder() { (void)hipFree(p); }
    } guard{d_order};
    uint8_t* d_pos_dims = nullptr;
    struct FreeDims {
        uint8_t** p;
        ~FreeDims() { (void)hipFree(*p); }
    } guard_dims{&d_pos_dims};
    if (split == KD_SPLIT_WIDEST) {
        try {
            t->pos_dims.resize(size_t(N));
        } catch (...) {
            return set_error(KD_ENOMEM, "kd_build: host allocation");
        }
        KD_HIP(hipMalloc(&d_pos_dims, size_t(N)));
        KD_HIP(hipMalloc(&t->d_dims, size_t(N) + 2));
    }
    s = build_level_order_device(points, N, dim, d_order, st, d_pos_dims);
    if (s != KD_OK) {
        if (t->d_dims) (void)hipFree(t->d_dims);
        return s;
    }
    hipError_t e = hipMalloc(&t->d_nodes, node_buffer_bytes(dim, N));
    if (e != hipSuccess) {
        if (t->d_dims) (void)hipFree(t->d_dims);
        return hip_error(e, "kd_build: nodes");
    }
    e = hipMalloc(&t->d_boxes, box_buffer_bytes(dim, N));
    if (e != hipSuccess) {
        (void)hipFree(t->d_nodes);
        if (t->d_dims) (void)hipFree(t->d_dims);
        return hip_error(e, "kd_build: boxes");
    }
    s = pack_tree_device(points, d_order, N, dim, t->d_nodes, static_cast<float*>(t->d_boxes), st, d_pos_dims,
                         t->d_dims);
    float root_box[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (s == KD_OK) {
        e = hipMemcpyAsync(t->order.data(), d_order, size_t(N) * 4, hipMemcpyDeviceToHost, st);
        // the root's box is the bounding box of all points
        if (e == hipSuccess)
            e = hipMemcpyAsync(root_box, static_cast<float*>(t->d_boxes) + box_words(dim), box_words(dim) * 4,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && d_pos_dims)
            e = hipMemcpyAsync(t->pos_dims.data(), d_pos_dims, size_t(N), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) s = hip_error(e, "kd_build: read back");
    }
    if (s != KD_OK) {
        (void)hipFree(t->d_nodes);
        (void)hipFree(t->d_boxes);
        if (t->d_dims) (void)hipFree(t->d_dims);
        return s;
    }
    for (int j = 0; j < dim; ++j) {
        t->lo[j] = root_box[j];
        t->hi[j] = root_box[box_words(dim) / 2 + j];
    }
    *out = t.release();
    return KD_OK;
}

kd_status kd_build_order_host(const float* host_points, int64_t N, int dim, int32_t* host_order) {
    if (N < 0 || N > KD_MAX_POINTS) return set_error(KD_EINVAL, "kd_build_order_host: N out of range [0, 2^30 - 1]");
    if (dim < 1 || dim > 8) return set_error(KD_EINVAL, "kd_build_order_host: dim must be in 1..8");
    if (N > 0 && (!host_points || !host_order)) return set_error(KD_EINVAL, "kd_build_order_host: NULL pointer");
    try {
        build_level_order(host_points, N, dim, host_order, 0);
    } catch (const std::exception& e) {
        return set_error(KD_ENOMEM, std::string("kd_build_order_host: ") + e.what());
    }
    return KD_OK;
}

kd_status kd_tree_free(kd_tree t) {
    if (!t) return KD_OK;
    if (t->d_nodes) (void)hipFree(t->d_nodes);
    if (t->d_boxes) (void)hipFree(t->d_boxes);
    if (t->d_dims) (void)hipFree(t->d_dims);
    delete t;
    return KD_OK;
}

kd_status kd_workspace_size(int64_t Q, int k, int flags, size_t* bytes) {
    if (!bytes) return set_error(KD_EINVAL, "kd_workspace_size: bytes is NULL");
    if (Q < 0 || Q >= (int64_t(1) << 31)) return set_error(KD_EINVAL, "kd_workspace_size: Q out of range [0, 2^31)");
    if (k < 1 || k > KD_MAX_K) return set_error(KD_EINVAL, "kd_workspace_size: k out of range [1, 64]");
    if (flags & ~KD_WS_LEARNED) return set_error(KD_EINVAL, "kd_workspace_size: unknown flags");
    // upper bound over dim (D = 4 has the largest records) and launch options
    // (sorted, with the hand-off rows)
    size_t b = 0;
    for (int dim = 2; dim <= 4; ++dim)
        b = std::max(b, query_scratch_bytes(Q, dim, true, (flags & KD_WS_LEARNED) != 0, true));
    *bytes = Q == 0 ? 0 : b;
    return KD_OK;
}

kd_status kd_tree_info(kd_tree t, int64_t* N, int* dim, float* lo4, float* hi4) {
    if (!t) return set_error(KD_EINVAL, "kd_tree_info: tree is NULL");
    if (N) *N = t->N;
    if (dim) *dim = t->dim;
    if (lo4) std::memcpy(lo4, t->lo, sizeof(t->lo));
    if (hi4) std::memcpy(hi4, t->hi, sizeof(t->hi));
    return KD_OK;
}

kd_status kd_tree_dims(kd_tree t, uint8_t* host_dims, int* split) {
    if (!t) return set_error(KD_EINVAL, "kd_tree_dims: tree is NULL");
    if (split) *split = t->split;
    if (!host_dims || t->N == 0) return KD_OK;
    if (t->split == KD_SPLIT_WIDEST) {
        std::memcpy(host_dims, t->pos_dims.data(), size_t(t->N));
    } else {
        for (int64_t pos = 0; pos < t->N; ++pos) {
            int lvl = 0;
            while ((int64_t(2) << lvl) <= pos + 1) ++lvl;  // floor(log2(pos + 1))
            host_dims[pos] = uint8_t(lvl % t->dim);
        }
    }
    return KD_OK;
}

kd_status kd_tree_order(kd_tree t, int32_t* host_order) {
    if (!t) return set_error(KD_EINVAL, "kd_tree_order: tree is NULL");
    if (t->N > 0 && !host_order) return set_error(KD_EINVAL, "kd_tree_order: host_order is NULL");
    if (t->N > 0) std::memcpy(host_order, t->order.data(), size_t(t->N) * sizeof(int32_t));
    return KD_OK;
}

kd_status kd_fcp(kd_tree t, const float* queries, int64_t Q, float maxRadius, int32_t* out_idx, float* out_d2,
                 kd_stream stream) {
    return knn_entry(t, queries, Q, 1, maxRadius, out_idx, out_d2, nullptr, nullptr, stream, "kd_fcp");
}

kd_status kd_knn(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius, int32_t* out_idx,
                 float* out_d2, kd_stream stream) {
    return knn_entry(t, queries, Q, k, maxRadius, out_idx, out_d2, nullptr, nullptr, stream, "kd_knn");
}

kd_status kd_knn_ex(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius, int32_t* out_idx,
                    float* out_d2, uint32_t* visited, const kd_opts* opts, kd_stream stream) {
    return knn_entry(t, queries, Q, k, maxRadius, out_idx, out_d2, visited, opts, stream, "kd_knn_ex");
}

namespace {
kd_status range_entry(kd_tree t, const float* in, int64_t Q, bool box, float maxRadius, int cap, int32_t* out_idx,
                      float* out_d2, uint32_t* out_count, uint32_t* visited, int flags, kd_stream stream,
                      const char* fn) {
    std::string f(fn);
    if (flags & ~KD_RANGE_BOXES) return set_error(KD_EINVAL, f + ": unknown flags");
    if (Q < 0 || Q >= (int64_t(1) << 31)) return set_error(KD_EINVAL, f + ": Q out of range [0, 2^31)");
    if (cap < 0 || cap > KD_MAX_K) return set_error(KD_EINVAL, f + ": cap out of range [0, 64]");
    if (!box && (std::isnan(maxRadius) || maxRadius < 0.0f))
        return set_error(KD_EINVAL, f + ": maxRadius must be >= 0 or +inf");
    if (!t) return set_error(KD_EINVAL, f + ": tree is NULL");
    if (Q > 0 && !in) return set_error(KD_EINVAL, f + (box ? ": boxes is NULL" : ": queries is NULL"));
    if (Q > 0 && !out_count) return set_error(KD_EINVAL, f + ": out_count is NULL");
    if (Q > 0 && cap > 0 && !out_idx) return set_error(KD_EINVAL, f + ": out_idx is NULL");
    if (Q == 0) return KD_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (t->N == 0) {
        hipLaunchKernelGGL(fill_zero_u32, dim3(unsigned((Q + 255) / 256)), dim3(256), 0, st, out_count, Q);
        KD_HIP(hipGetLastError());
        if (visited) {
            hipLaunchKernelGGL(fill_zero_u32, dim3(unsigned((Q + 255) / 256)), dim3(256), 0, st, visited, Q);
            KD_HIP(hipGetLastError());
        }
        if (cap > 0) {
            const int64_t n = Q * cap;
            hipLaunchKernelGGL(fill_empty, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, out_idx,
                               box ? nullptr : out_d2, n);
            KD_HIP(hipGetLastError());
        }
        return KD_OK;
    }
    const float R2 = box ? 0.0f : maxRadius * maxRadius;  // binary32 product; +inf stays +inf
    return run_range(t, in, Q, box, R2, cap, cap > 0 ? out_idx : nullptr, box || cap == 0 ? nullptr : out_d2,
                     out_count, visited, (flags & KD_RANGE_BOXES) == 0, stream);
}
}  // namespace

kd_status kd_radius_search(kd_tree t, const float* queries, int64_t Q, float maxRadius, int cap, int32_t* out_idx,
                           float* out_d2, uint32_t* out_count, uint32_t* visited, int flags, kd_stream stream) {
    return range_entry(t, queries, Q, false, maxRadius, cap, out_idx, out_d2, out_count, visited, flags, stream,
                       "kd_radius_search");
}

kd_status kd_box_search(kd_tree t, const float* boxes, int64_t Q, int cap, int32_t* out_idx, uint32_t* out_count,
                        uint32_t* visited, int flags, kd_stream stream) {
    return range_entry(t, boxes, Q, true, 0.0f, cap, out_idx, nullptr, out_count, visited, flags, stream,
                       "kd_box_search");
}

const char* kd_status_str(kd_status s) {
    switch (s) {
        case KD_OK: return "KD_OK";
        case KD_EINVAL: return "KD_EINVAL: invalid argument";
        case KD_ENOMEM: return "KD_ENOMEM: out of memory";
        case KD_EHIP: return "KD_EHIP: HIP runtime error";
        case KD_EUNSUPPORTED: return "KD_EUNSUPPORTED: not supported";
    }
    return "unknown kd_status";
}

const char* kd_last_error(void) { return g_last_error.c_str(); }

kd_status kd_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing_on = on != 0;
    return KD_OK;
}

kd_status kd_timing_collect(const char* kernel, double* total_ms, int64_t* launches) {
    if (!kernel || !total_ms || !launches) return set_error(KD_EINVAL, "kd_timing_collect: NULL argument");
    std::vector<TimedLaunch> all;
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        std::vector<TimedLaunch> keep;
        for (auto& t : g_timed) (t.kernel == kernel ? all : keep).push_back(t);
        g_timed.swap(keep);
    }
    double ms = 0;
    int64_t n = 0;
    kd_status st = KD_OK;
    for (auto& t : all) {
        if (st == KD_OK) {
            hipError_t e = hipEventSynchronize(t.b);
            float m = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&m, t.a, t.b);
            if (e != hipSuccess) st = hip_error(e, "kd_timing_collect");
            ms += m;
            ++n;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    *total_ms = ms;
    *launches = n;
    return st;
}

const char* kd_version(void) { return "kdtree-gfx950 0.1"; }

}  // extern "C"
