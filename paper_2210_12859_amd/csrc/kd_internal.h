// kd_internal.h -- internal declarations shared by the libkdtree sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kdtree.h"

namespace kd {

// Node record in the array-of-structures layout: the D coordinates followed by
// the caller index, one record per level-order position, padded to 16 bytes
// (D = 2, 3) or 32 bytes (D = 4) so that one aligned vector load fetches a
// whole node.
template <int D>
struct alignas(16) NodeRec {
    float c[D];
    int32_t idx;
};

// Tree node record: RW = rec_words(D) 32-bit words per level-order position:
// w[0..D-1] the coordinates, then (D = 2, 4) w[D] the caller index, then the
// split values of the nearest ancestors, parent first (the coordinate of the
// ancestor's point in that ancestor's split dimension).  Ancestor splits let
// a lane resolve "return to parent" steps of the traversal from the record it
// already holds, without loading the parent.
//   D = 2: 16 bytes {x, y, index, parent split}
//   D = 3: 16 bytes {x, y, z, parent split}; the caller index lives in a
//          separate int32 array after the records (node buffer = records
//          [N + 2], then indices [N + 2]), read only when a point can enter
//          the k-best list, so a traversal step is one dwordx4 load
//   D = 4: 32 bytes {x, y, z, w, index, 3 ancestor splits}
#ifndef KD_IDX_SPLIT_D3
#define KD_IDX_SPLIT_D3 1
#endif
#ifndef KD_REC_WORDS_D3
#define KD_REC_WORDS_D3 8
#endif
constexpr bool rec_has_idx(int D) { return !(D == 3 && KD_IDX_SPLIT_D3); }
constexpr int rec_words(int D) { return D == 2 ? 4 : (D == 3 ? (KD_IDX_SPLIT_D3 ? 4 : KD_REC_WORDS_D3) : 8); }
constexpr int rec_ancestors(int D) { return rec_words(D) - D - (rec_has_idx(D) ? 1 : 0); }
// node buffer bytes for N points (records, then the index array if separate)
inline size_t node_buffer_bytes(int D, int64_t N) {
    const size_t recs = size_t(N + 2) * 4 * size_t(rec_words(D));
    return rec_has_idx(D) ? recs : recs + size_t(N + 2) * 4;
}

template <int D>
struct alignas(4 * rec_words(D)) TreeRec {
    uint32_t w[rec_words(D)];
};

// Subtree bounding boxes, one per node id: the per-dimension minimum of the
// points of the node's subtree at words 0..D-1, the maximum at words
// box_words(D)/2 .. box_words(D)/2 + D-1 (D = 3 pads both halves to 4 words,
// so a box is two aligned dwordx4 loads).
constexpr int box_words(int D) { return D == 2 ? 4 : 8; }
inline size_t box_buffer_bytes(int D, int64_t N) { return size_t(N + 2) * 4 * size_t(box_words(D)); }
// Box tests are made for subtrees spanning at least this many levels (near the
// leaves a test costs about as much as the few nodes it could skip).
#ifndef KD_BOX_MIN_HEIGHT
#define KD_BOX_MIN_HEIGHT 3
#endif
// First node id whose subtree spans fewer than KD_BOX_MIN_HEIGHT levels
// (ids of depth <= levels - KD_BOX_MIN_HEIGHT, levels = floor(log2 N) + 1).
inline int32_t box_id_limit(int64_t N) {
    int levels = 0;
    while (levels < 31 && (int64_t(1) << levels) <= N) ++levels;
    const int e = levels - KD_BOX_MIN_HEIGHT + 1;
    return e <= 0 ? 1 : int32_t(1) << e;  // N < 2^30: e <= 28
}

// Tuned launch parameters kept with a tree (filled by kd_autotune).
struct TuneEntry {
    int k_template;  // compiled list size
    kd_opts opts;
};

struct Workspace;

}  // namespace kd

struct kd_tree_s {
    int64_t N = 0;
    int dim = 0;
    int device = 0;
    int split = 0;                 // KD_SPLIT_LEVEL or KD_SPLIT_WIDEST
    float lo[4] = {0, 0, 0, 0};
    float hi[4] = {0, 0, 0, 0};
    void* d_nodes = nullptr;       // node buffer: TreeRec<dim>[N + 2], record of node id i at index i
                                   // (+ int32 index[N + 2] when the record holds no index)
    void* d_boxes = nullptr;       // float[N + 2][box_words(dim)]: bounding box of the points of the
                                   // subtree of node id i (lows, then highs) at index i
    uint8_t* d_dims = nullptr;     // trees with stored split dimensions: uint8[N + 2] by node id, bits
                                   // 2m..2m+1 = split dimension of the ancestor m levels up (m = 0:
                                   // the node); NULL: the dimension of node id i is floor(log2 i) mod dim
    std::vector<int32_t> order;    // host copy: order[pos] = caller index
    std::vector<uint8_t> pos_dims; // host copy of the stored dimensions by position (else empty)
    std::mutex tune_mu;
    std::vector<kd::TuneEntry> tuned;
};

namespace kd {

// ---- errors -------------------------------------------------------------
kd_status set_error(kd_status s, const std::string& msg);
kd_status hip_error(hipError_t e, const char* what);
#define KD_HIP(call)                                                \
    do {                                                            \
        hipError_t _e = (call);                                     \
        if (_e != hipSuccess) return ::kd::hip_error(_e, #call);    \
    } while (0)

// ---- host builder (kd_build_host.cpp) -------------------------------------
int64_t left_subtree_size(int64_t n);
// order[pos] = caller index; threads <= 0 picks the hardware count.
void build_level_order(const float* pts, int64_t N, int dim, int32_t* order, int threads);

// ---- tuned options (kd_autotune.cpp) ----------------------------------------
bool tuned_opts(kd_tree t, int K, kd_opts* out);

// ---- device info --------------------------------------------------------
struct DeviceInfo {
    int cus = 256;
    int lds_bytes = 160 * 1024;
    int xcds = 8;
};
const DeviceInfo& device_info(int device);

// ---- per-stream scratch (kd_api.cpp) --------------------------------------
// Returns a device buffer of at least `bytes`, private to (device, stream).
// Calls on one stream are ordered, so reuse across calls is safe.
kd_status scratch(kd_stream stream, size_t bytes, void** out);
// A second such buffer per (device, stream), for data a call keeps across
// the launches that use scratch() (the range queries' counts and scan totals).
kd_status aux_scratch(kd_stream stream, size_t bytes, void** out);

// ---- kernel timing hook (kd_api.cpp) --------------------------------------
// When enabled, launches of the named kernel are bracketed by hipEvents on
// the stream they run on; kd_timing_collect sums the elapsed times.
bool timing_enabled();
kd_status timing_begin(hipStream_t st, hipEvent_t* ev);
kd_status timing_end(hipStream_t st, hipEvent_t ev0, const char* kernel);

// ---- query pipeline (kd_traverse.hip) -------------------------------------
struct QueryPlan {
    int k = 1;
    int K = 1;          // compiled list size >= k
    float R2 = 0;
    int block = 256;
    int lds_levels = 0;   // top tree levels staged in LDS (plain queries), 0 = none
    int sort_bits = 32;
    int waves_per_cu = 8;
    int heavy_trips = 0;  // trip budget before the cooperative hand-off, 0 = none
    bool heavy_default = true;  // the budget was left at its default
    int prune = 0;        // kd_opts.prune: 0 default, 1 split planes, 2 subtree boxes
};
int k_template(int k);

// One job of a batched call, as the device sees it.  Jobs of one (dim, K)
// class are laid out back to back in a class slot space.
struct BatchJob {
    const void* nodes;       // TreeRec<D>[N + 2], record of node id i at index i
    const float* boxes;      // subtree bounding boxes of the tree (see box_words)
    int32_t box_below;       // boxes are tested for node ids below this
    const float* queries;    // caller [Q][D]
    int32_t* out_idx;        // caller [Q][k]
    float* out_d2;           // caller [Q][k] or NULL
    float lo[4], scale[4];   // Morton normalisation over the tree's bounding box
    int32_t N;
    int32_t k;
    float R2;
    uint32_t slot_base;      // first class slot of the job
    uint32_t Q;
    int32_t vec_store;
    int32_t learned;         // starts from the initial radius in worst0 (3-D jobs with a model)
};

// A batched job whose initial radii come from a radius model, as the MLP
// kernel sees it: the job's class records [slot_base, slot_base + Q) (each
// job's records are contiguous after the class sort) are tiles
// tile_base .. tile_base + ceil(Q / 64) - 1 of the class.
struct MlpJob {
    const float* P;          // model parameters (4481 floats)
    float lo[3], inv[3];     // input normalisation
    float margin;
    float R2;
    uint32_t slot_base, Q, tile_base, pad;
};
struct BatchLearned {
    const MlpJob* jobs;      // device table, ascending tile_base
    int njobs;
    uint32_t ntiles;
    float* worst0;           // [class records]
};

// Learned-radius request: initial squared radius per query from the MLP
// (params != NULL) or from caller radii r0 (caller order).
struct LearnedSpec {
    const float* params;  // device, 4481 floats, or NULL
    float lo[3], inv[3];
    float margin;
    const float* r0;      // device [Q] caller order (when params == NULL)
    uint8_t* fb_flag;     // device [Q] caller order, nullable
};
// Batched class pipeline (kd_sort.hip, kd_traverse.hip)
size_t batch_sort_scratch_bytes(int64_t n);
kd_status batch_sort(const BatchJob* d_jobs, int njobs, int dim, uint32_t n, int sort_bits, void* ws,
                     hipStream_t st, const uint32_t** perm_out);
// learned (nullable): initial radii of the class's 3-D jobs with a model;
// heavy_rows (nullable): [batch_heavy_cap][2] hand-off list (NULL: no hand-off)
kd_status run_batch_class(const BatchJob* d_jobs, int njobs, int dim, int K, uint32_t n, const uint32_t* perm,
                          void* recs, uint32_t* counters, const QueryPlan& plan, int device, hipStream_t st,
                          const BatchLearned* learned, int32_t* heavy_rows);
size_t batch_rec_bytes();
size_t batch_cursor_bytes();  // hand-off count and work cursors of one class launch
uint32_t batch_heavy_cap(int device);  // hand-off list entries of one class launch
// Morton reorder of query slots (kd_sort.hip)
size_t sort_scratch_bytes(int64_t Q, int dim);
// Stable LSD radix sort of n (key, value) pairs on key bits [0, bits), 8 bits
// per pass, ping-ponging between (k0, v0) and (k1, v1); *in_second tells
// which pair holds the result.  ws holds sort_pairs_scratch_bytes(n).
size_t sort_pairs_scratch_bytes(uint32_t n);
kd_status sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t n, int bits, void* ws,
                     hipStream_t st, bool* in_second);
// Canonical tree on the device (kd_build_gpu.hip): d_order[pos] = caller
// index of the point at level-order position pos, for device points [N][dim].
// d_pos_dims non-NULL: the widest-extent rule, each position's split
// dimension written there (uint8 [N]); NULL: the dimension by level.
kd_status build_level_order_device(const float* d_pts, int64_t N, int dim, int32_t* d_order, hipStream_t st,
                                   uint8_t* d_pos_dims = nullptr);
// Node records and subtree boxes from device points and order (kd_build_gpu.hip);
// with stored dimensions (d_pos_dims by position) the records' ancestor splits
// follow them and d_dims (uint8 [N + 2], by node id) receives the packed
// dimensions of each node and its three nearest ancestors.
kd_status pack_tree_device(const float* d_pts, const int32_t* d_order, int64_t N, int dim, void* d_nodes,
                           float* d_boxes, hipStream_t st, const uint8_t* d_pos_dims = nullptr,
                           uint8_t* d_dims = nullptr);
// *ok = no NaN or infinity among the N * dim device floats (synchronises).
kd_status check_points_finite(const float* d_pts, int64_t N, int dim, hipStream_t st, bool* ok);
// device scratch of one kd_knn-family call (kd_traverse.hip)
size_t query_scratch_bytes(int64_t Q, int dim, bool sorted, bool learned, bool handoff);
// Writes the queries as traversal records (NodeRec<dim>[Q]) into sq, in
// Morton order on the top sort_bits bits (0: caller order), and clears
// zero[0..nzero) on the way.  ws holds sort_scratch_bytes(Q, dim) when sort_bits > 0.
kd_status reorder_queries(kd_tree t, const float* queries, int64_t Q, int sort_bits, void* ws, void* sq,
                          uint32_t* zero, uint32_t nzero, hipStream_t st);
// A caller-provided device scratch region of `bytes` bytes that replaces the
// per-stream buffer; a call whose scratch does not fit fails with KD_EINVAL
// before any launch.  Calls given one records no timing events.
struct FixedScratch {
    void* ptr;
    size_t bytes;
};
// Range queries (kd_traverse.hip): box = false, queries_or_boxes holds
// float [Q][dim] points and R2 the squared radius; box = true, it holds float
// [Q][2][dim] boxes.  Writes out_count[Q] and, for cap > 0, out_idx[Q][cap]
// (and out_d2[Q][cap] for radius queries when given), and visited[Q] (the
// entered nodes) when given.  Q >= 1, N >= 1.  planes_only: no subtree box
// tests (split planes only).  Fill mode (fill_idx non-NULL; cap 0 and
// planes_only): every point in range of caller row r is also written to
// fill_idx[fill_off[r] + its rank in traversal order].
kd_status run_range(kd_tree t, const float* queries_or_boxes, int64_t Q, bool box, float R2, int cap,
                    int32_t* out_idx, float* out_d2, uint32_t* out_count, uint32_t* visited, bool planes_only,
                    kd_stream stream, const int64_t* fill_off = nullptr, int32_t* fill_idx = nullptr);
kd_status run_knn(kd_tree t, const float* queries, int64_t Q, const QueryPlan& plan, int32_t* out_idx,
                  float* out_d2, uint32_t* visited, kd_stream stream, const LearnedSpec* learned = nullptr,
                  kd_stats* stats = nullptr, const FixedScratch* fixed = nullptr);

// ---- query entry helpers (kd_api.cpp) --------------------------------------
// Validation shared by the query entry points (nothing enqueued on error).
kd_status check_query_args_public(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius,
                                  const int32_t* out_idx, const char* fn);
// Launch plan for (tree, k) from opts, else the tree's tuned options, else defaults.
kd_status resolve_plan_public(kd_tree t, int k, float maxRadius, const kd_opts* o, QueryPlan& p);
// Validated plain kNN: empty trees answered without traversal, else run_knn.
kd_status knn_entry(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius, int32_t* out_idx,
                    float* out_d2, uint32_t* visited, const kd_opts* opts, kd_stream stream, const char* fn,
                    const FixedScratch* fixed = nullptr);

// ---- result checksum (kd_batch.cpp) -----------------------------------------
// XORs into *h an order-independent, position-sensitive 64-bit hash of n
// result slots (index, and d2 bits when d2 is not NULL); the autotuners
// check with it that every candidate writes the same results.
hipError_t launch_output_checksum(const int32_t* idx, const float* d2, int64_t n, uint64_t salt,
                                  unsigned long long* h, hipStream_t st);

// ---- radius models (kd_model.cpp) -------------------------------------------
// The model's device parameters, normalisation and margin (R2, slots and tiles
// left for the caller).
kd_status model_view(kd_model m, MlpJob* out);

// ---- MLP kernels (kd_mlp.hip) ---------------------------------------------
constexpr int MLP_NPARAM = 4481;
// Adam hyper-parameters of the trainer (float32 values)
constexpr float MLP_ADAM_BETA1 = 0.9f, MLP_ADAM_BETA2 = 0.999f, MLP_ADAM_EPS = 1e-8f;
hipError_t launch_mlp_worst0(const float* P, const float* lo, const float* inv, float margin, float R2,
                             const void* sq, uint32_t Q, float* worst0, hipStream_t st);
// worst0 for the batched class records (32 bytes: x, y, z, w, row, job, pad)
// of the jobs in the table; other records are left untouched
hipError_t launch_mlp_worst0_jobs(const MlpJob* jobs, int njobs, uint32_t ntiles, const void* recs, float* worst0,
                                  hipStream_t st);
// worst0 for caller-layout queries [n][3], in caller order (recs: n x 16 bytes of scratch)
hipError_t launch_mlp_worst0_rows(const float* P, const float* lo, const float* inv, float margin, float R2,
                                  const float* queries, uint32_t n, void* recs, float* worst0, hipStream_t st);
hipError_t launch_mlp_predict(const float* P, const float* lo, const float* inv, const float* qs, uint32_t n,
                              float* y, hipStream_t st);
hipError_t launch_mlp_fwd_bwd(const float* P, const float* lo, const float* inv, const float* qs, const float* t,
                              const uint32_t* idx, uint32_t b0, uint32_t batch, float* part, float* part_loss,
                              hipStream_t st);
hipError_t launch_mlp_reduce_adam(const float* part, const float* part_loss, int nparts, uint32_t batch, float* P,
                                  float* m, float* v, int step, float lr, float* grad, float* loss, hipStream_t st);
hipError_t launch_knn_label(const float* d2, int k, uint32_t n, float* t, hipStream_t st);

}  // namespace kd
