// kd_traverse.hip -- stack-free fcp / kNN traversal kernels for gfx950, the
// cooperative hand-off, the batched and learned-radius variants, and the
// un-ordered range-query kernels (radius and box search, end of file).
//
// Each lane runs the two-integer state machine of the paper's Sec. 3.2 for
// one query: `curr` and `prev` alone decide where to go next.
//   * first visit (prev < curr, i.e. we came from the parent): process the
//     node -- squared distance, insertion into the k-best list, which may
//     shrink the search radius -- then step to the close child;
//   * second visit (prev == close child): step to the far child if its
//     subtree is still in range, else to the parent;
//   * third visit (prev == far child): step to the parent;
//   * the root stepping to its parent ends the traversal.
// The close child is the right child iff q[dim] - split > 0 (Sec. 3.2).  The
// far-range test is taken in squared form, fl(sd*sd) <= worst d2 of the list,
// non-strict: every point of the far subtree has d2 >= fl(sd*sd), so the test
// never prunes a point that could enter the list, ties included.
//
// Node ids inside the kernel are 1-based (id = array position + 1): children
// of i are 2i and 2i+1, the sibling of c is c^1, the parent is i>>1, and the
// root's parent is 0, which ends the traversal.  This is the paper's
// level-order layout with the index shifted by one.
//
// Several state-machine steps run per loop trip, always in the paper's order:
//   * a step onto a child that does not exist (id > N) and the bounce back
//     are resolved in place: the next node is the one the bounce would pick;
//   * a "return to parent" step is resolved with the parent's split value
//     stored in the current node's record (one level for D = 2 and 3, three
//     ancestors for D = 4), so a lane does not reload its parent to learn
//     which child it came from.
// The split dimension of a node is its level's (floor(log2 id) mod D), or,
// for trees that store it (the XD kernels), read from a byte per node that
// also holds the dimensions of its three nearest ancestors.
// The processed-node sequence therefore equals the paper's, and the ordered
// recursion's, node for node.
//
// MI355X mapping
//   * persistent grid sized to one round of resident workgroups; each
//     workgroup owns a contiguous range of the Morton-sorted queries (its
//     CU's L1 and its XCD's L2 hold that region of the tree), with bounded
//     stealing at the end;
//   * each wave pulls 64 queries at a time with one coalesced load and hands
//     them to idle lanes by cross-lane shuffle, so a lane restarts without a
//     memory round trip;
//   * a step loads one 16-byte record (D = 2, 3: one dwordx4) or a 32-byte
//     record (D = 4: two dwordx4 from one cache line); with D = 3 the caller
//     index is read from its own array, only for points that can enter the
//     k-best list;
//   * the k-best list lives in VGPRs as 64-bit keys (d2 bits << 32 | index),
//     so the lexicographic (d2, index) order is one unsigned compare (d2 >= 0,
//     and the bit pattern of a non-negative float is monotone); insertion is
//     a fixed, fully unrolled network behind a wave-uniform skip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <type_traits>

#include "kd_internal.h"


namespace kd {

namespace {

constexpr uint32_t SENT_IDX = 0x7fffffffu;

struct TravArgs {
    const void* nodes;       // TreeRec<D>[N + 2], record of node id i at index i
    const uint8_t* dims;     // stored split dimensions by node id (XD kernels), else NULL
    const float* boxes;      // [N + 2][box_words(D)] subtree bounding boxes (BOX kernels)
    int32_t box_below;       // boxes are tested for node ids below this (subtrees tall enough)
    int32_t lds_below;       // LDS kernels: records of node ids 1 .. lds_below-1 are staged in LDS
    uint32_t refill_min;     // idle lanes are refilled once at least this many are idle
    int32_t N;
    const void* sq;          // NodeRec<D>[Q]: queries in traversal order, .idx = caller row
    uint32_t Q;              // query slots
    int k;                   // requested k (<= K)
    float R2;                // fl32(maxRadius^2)
    int32_t* out_idx;        // [Q][k] caller order
    float* out_d2;           // [Q][k] or NULL
    uint32_t* visited;       // [Q] or NULL
    uint32_t* counter;       // [gridDim.x] per-workgroup range cursors, zero at launch
    int vec_store;           // outputs 16-byte aligned with k % 4 == 0: vector stores
    // learned-radius kernels
    const float* worst0;     // [Q] initial squared radius per slot
    const int32_t* start;    // [Q] node id the slot's initial-radius run starts from
    uint32_t* fb_count;      // queries restarted from R2 (nullable)
    unsigned long long* vis_total;  // entered nodes summed over the launch (nullable, learned kernels)
    uint8_t* fb_flag;        // [Q] caller order, 1 = restarted from R2 (nullable)
    // hand-off of long traversals to the cooperative kernel
    uint32_t heavy_trips;    // trip budget per query, 0 = none
    uint32_t heavy_cap;      // at most this many rows are handed off
    uint32_t* heavy_count;   // rows that asked for a hand-off (zero at launch; may exceed heavy_cap)
    int32_t* heavy_rows;     // [heavy_cap] caller rows handed off
};

// Wave votes on a lane predicate held as a lane mask (no round trip through
// a VGPR, as the int-argument forms take).
__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

__device__ __forceinline__ uint64_t make_key(float d2, int32_t idx) {
    return (uint64_t(__float_as_uint(d2)) << 32) | uint32_t(idx);
}

__device__ __forceinline__ float key_d2(uint64_t key) { return __uint_as_float(uint32_t(key >> 32)); }

// Sorted insertion of `key` (known to be < L[K-1]) into the ascending list L.
#ifndef KD_INSERT_MED3
#define KD_INSERT_MED3 1
#endif
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
    // the median-of-three form the compiler maps to one v_med3_u32
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    const uint32_t m = hi < c ? hi : c;
    return lo > m ? lo : m;
}

// Slot j becomes key clamped to [L[j-1], L[j]] (64-bit order).  Its high
// word (the d2 bits) is the median of the three high words, as the list is
// sorted; its low word (the index) follows the two 64-bit comparisons.
template <int K>
__device__ __forceinline__ void list_insert(uint64_t (&L)[K], uint64_t key) {
#if KD_INSERT_MED3
    const uint32_t khi = uint32_t(key >> 32), klo = uint32_t(key);
#pragma unroll
    for (int j = K - 1; j > 0; --j) {
        const bool lt_prev = key < L[j - 1];
        const bool lt_here = key < L[j];
        const uint32_t hi = med3_u32(uint32_t(L[j - 1] >> 32), khi, uint32_t(L[j] >> 32));
        const uint32_t lo = lt_prev ? uint32_t(L[j - 1]) : (lt_here ? klo : uint32_t(L[j]));
        L[j] = (uint64_t(hi) << 32) | lo;
    }
    {
        const bool lt0 = key < L[0];
        const uint32_t h0 = uint32_t(L[0] >> 32);
        L[0] = (uint64_t(khi < h0 ? khi : h0) << 32) | (lt0 ? klo : uint32_t(L[0]));
    }
#else
#pragma unroll
    for (int j = K - 1; j > 0; --j) {
        const bool lt_prev = key < L[j - 1];
        const bool lt_here = key < L[j];
        L[j] = lt_prev ? L[j - 1] : (lt_here ? key : L[j]);
    }
    L[0] = key < L[0] ? key : L[0];
#endif
}

// Split dimension of node id n (1-based) is level mod D with level =
// 31 - clz(n).  DimSel holds the one-hot flags dim == j (j = 1..D-1), read
// as bit clz(n) of compile-time patterns: no division on the step path.
constexpr uint32_t dim_pattern(int D, int j) {
    uint32_t p = 0;
    for (int c = 0; c < 32; ++c)
        if ((31 - c) % D == j) p |= 1u << c;
    return p;
}

template <int D>
struct DimSel {
    bool f[4];  // f[j]: dim == j (f[0] unused)
    DimSel() = default;
    // a stored dimension d (0 .. D-1)
    static __device__ __forceinline__ DimSel of(uint32_t d) {
        DimSel r;
        r.f[0] = false;
#pragma unroll
        for (int j = 1; j < 4; ++j) r.f[j] = j < D && d == uint32_t(j);
        return r;
    }
    __device__ __forceinline__ explicit DimSel(int32_t id) {
        const uint32_t c = uint32_t(__builtin_clz(uint32_t(id)));  // id >= 1
        f[0] = false;
#pragma unroll
        for (int j = 1; j < 4; ++j) f[j] = j < D ? __builtin_amdgcn_ubfe(dim_pattern(D, j), c, 1) != 0 : false;
    }
    // v[(dim - I) mod D] as a chain of D - 1 selects between values (the
    // values are passed one by one: a select between elements of a local
    // array is turned into an indexed access, which lives in LDS/scratch)
    template <int J>
    static __device__ __forceinline__ float pick(float v0, float v1, float v2, float v3) {
        return J == 0 ? v0 : (J == 1 ? v1 : (J == 2 ? v2 : v3));
    }
    template <int I>
    __device__ __forceinline__ float rot(float v0, float v1, float v2, float v3) const {
        float r = pick<(D - I % D) % D>(v0, v1, v2, v3);
        if (D > 1) r = f[1] ? pick<(1 - I % D + D) % D>(v0, v1, v2, v3) : r;
        if (D > 2) r = f[2] ? pick<(2 - I % D + D) % D>(v0, v1, v2, v3) : r;
        if (D > 3) r = f[3] ? pick<(3 - I % D + D) % D>(v0, v1, v2, v3) : r;
        return r;
    }
    template <int I>
    __device__ __forceinline__ float rot(const float (&v)[D]) const {
        return rot<I>(v[0], v[1], D > 2 ? v[D > 2 ? 2 : 0] : 0.0f, D > 3 ? v[D > 3 ? 3 : 0] : 0.0f);
    }
};

// Split dimension of node `id` at `up` levels above it (0: the node): by
// level, or (XD, trees with stored dimensions) from the node's dimension
// byte db, which holds 2 bits for the node and each of its three nearest
// ancestors.  rot<0> of the result picks that node's split coordinate.
template <int D, bool XD, int UP>
__device__ __forceinline__ DimSel<D> split_dim(int32_t id, uint32_t db) {
    if constexpr (XD) return DimSel<D>::of((db >> (2 * UP)) & 3u);
    else return DimSel<D>(id >> UP);
}

// Whole-record loads: one or two dwordx4 from one aligned record.
template <int D>
__device__ __forceinline__ void load_tree(const TreeRec<D>* p, float (&c)[D], int32_t& idx,
                                          float (&anc)[rec_ancestors(D) > 0 ? rec_ancestors(D) : 1]) {
    constexpr int RW = rec_words(D);
    uint32_t w[8];
    const uint4 lo = reinterpret_cast<const uint4*>(p)[0];
    w[0] = lo.x; w[1] = lo.y; w[2] = lo.z; w[3] = lo.w;
    if (RW == 8) {
        const uint4 hi = reinterpret_cast<const uint4*>(p)[1];
        w[4] = hi.x; w[5] = hi.y; w[6] = hi.z; w[7] = hi.w;
    }
    constexpr int A0 = D + (rec_has_idx(D) ? 1 : 0);
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = __uint_as_float(w[j]);
    idx = rec_has_idx(D) ? int32_t(w[D]) : 0;
    anc[0] = 0.0f;
#pragma unroll
    for (int j = 0; j < rec_ancestors(D); ++j) anc[j] = __uint_as_float(w[A0 + j]);
}

// Whole-record load at a wave-uniform node id through the scalar data cache
// (constant address space: the tree is read-only for the whole launch).
template <int D>
__device__ __forceinline__ void load_tree_uniform(const TreeRec<D>* g1, int32_t id, float (&c)[D], int32_t& idx) {
    typedef __attribute__((address_space(4))) const uint32_t CWord;
    const CWord* w = (const CWord*)(g1 + __builtin_amdgcn_readfirstlane(id));
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = __uint_as_float(w[j]);
    idx = rec_has_idx(D) ? int32_t(w[D]) : 0;
}

// Lower bound of the squared distance from q to every point of the subtree
// of node id `id`, from the subtree's bounding box.  Per dimension the offset
// is q - low below the box, q - high above it, else 0; the squares are summed
// in the order of the point distance, without contraction.  Rounding is
// monotonic, so for each point p of the box |fl(q - p)| >= |offset| per
// dimension and the point's d2 is >= this sum: a subtree whose bound exceeds
// the current k-th distance holds no point of the result.
template <int D>
__device__ __forceinline__ float box_d2(const float* __restrict__ boxes, int32_t id, const float (&q)[D]) {
    constexpr int H = box_words(D) / 2;
    const uint4* p = reinterpret_cast<const uint4*>(boxes + int64_t(id) * box_words(D));
    float w[8];
    const uint4 a = p[0];
    w[0] = __uint_as_float(a.x); w[1] = __uint_as_float(a.y); w[2] = __uint_as_float(a.z); w[3] = __uint_as_float(a.w);
    if (box_words(D) == 8) {
        const uint4 b = p[1];
        w[4] = __uint_as_float(b.x); w[5] = __uint_as_float(b.y); w[6] = __uint_as_float(b.z); w[7] = __uint_as_float(b.w);
    }
    float o[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const float below = q[j] - w[j];      // < 0 when q is below the box
        const float above = q[j] - w[H + j];  // > 0 when q is above it
        o[j] = below < 0.0f ? below : (above > 0.0f ? above : 0.0f);
    }
    float d2 = o[0] * o[0];
#pragma unroll
    for (int j = 1; j < D; ++j) d2 = d2 + o[j] * o[j];
    return d2;
}

// Caller-index array of a node buffer whose records hold no index.
template <int D>
__device__ __forceinline__ const int32_t* node_ids(const TreeRec<D>* g1, int32_t N) {
    return rec_has_idx(D) ? nullptr : reinterpret_cast<const int32_t*>(g1 + (int64_t(N) + 2));
}

// Query records (16 bytes for D <= 3, 32 for D = 4).
template <int D>
__device__ __forceinline__ NodeRec<D> load_query(const NodeRec<D>* p) {
    const uint4 lo = reinterpret_cast<const uint4*>(p)[0];
    NodeRec<D> r;
    const uint32_t w[4] = {lo.x, lo.y, lo.z, lo.w};
    if (D < 4) {
#pragma unroll
        for (int j = 0; j < D; ++j) r.c[j] = __uint_as_float(w[j]);
        r.idx = int32_t(w[D < 4 ? D : 0]);
    } else {
#pragma unroll
        for (int j = 0; j < D; ++j) r.c[j] = __uint_as_float(w[j]);
        r.idx = int32_t(reinterpret_cast<const uint4*>(p)[1].x);
    }
    return r;
}

template <int D>
__device__ __forceinline__ NodeRec<D> shfl_rec(const NodeRec<D>& r, int src) {
    NodeRec<D> o;
#pragma unroll
    for (int j = 0; j < D; ++j) o.c[j] = __shfl(r.c[j], src);
    o.idx = __shfl(r.idx, src);
    return o;
}

// Fused "return to parent" levels per loop trip, at most the ancestor splits
// a record holds (D = 2, 3: one; D = 4: three).  On 4-D uniform data three
// levels beat one by 7-9 %.
#ifndef KD_FUSED_LEVELS
#define KD_FUSED_LEVELS 3
#endif
constexpr int fused_levels(int D) { return KD_FUSED_LEVELS < rec_ancestors(D) ? KD_FUSED_LEVELS : rec_ancestors(D); }

// Per-lane query state: the two node ids of the state machine (1-based),
// the split dimension of `curr` (implied by its level, tracked as the lane
// moves), the query and its k-best list.
//
// Learned-radius lanes start from the squared radius worst0 <= R2 instead
// of R2 (the list's sentinel entries carry worst0).  A lane that ends with
// fewer than k points found inside worst0 < R2 restarts in place from R2, so
// every result equals the plain traversal's.
template <int D, int K>
struct Lane {
    float q[D];
    uint64_t L[K];
    int32_t curr, prev;
    int32_t stop;      // the traversal ends on stepping to this node: 0 (root's parent), or the
                       // parent of the start node of a learned initial-radius run
    int32_t row;
    uint32_t vis;
    uint32_t t0;       // the wave's trip count when the current query started
    float w0;          // initial squared radius of the current run
    bool fell_back;    // the learned run found < k points and was restarted
    bool far_entry;    // the last step moved into a far child
};

template <int D, int K>
__device__ __forceinline__ void lane_reset(Lane<D, K>& s, int k, float w0) {
    s.w0 = w0;
    // Slots beyond k hold the smallest key so the list's worst entry is the
    // k-th real one; real keys are >= 0 and never move in front of them.
    const uint64_t sent = make_key(w0, SENT_IDX);
#pragma unroll
    for (int j = 0; j < K; ++j) s.L[j] = (j < K - k) ? uint64_t(0) : sent;
    s.curr = 1;   // root
    s.prev = 0;   // the root's parent
    s.stop = 0;
    s.far_entry = false;
}

template <int D, int K, bool LEARNED>
__device__ __forceinline__ void lane_start(Lane<D, K>& s, const TravArgs& a, const NodeRec<D>& qr, float w0,
                                           uint32_t wtrip = 0, int32_t start = 1) {
#pragma unroll
    for (int j = 0; j < D; ++j) s.q[j] = qr.c[j];
    s.row = qr.idx;
    s.vis = 0;
    s.t0 = wtrip;
    s.fell_back = false;
    lane_reset<D, K>(s, a.k, LEARNED ? w0 : a.R2);
    if (LEARNED) {
        // the initial-radius run covers the subtree of the start node only
        s.curr = start;
        s.prev = start >> 1;
        s.stop = start >> 1;
    }
}

// A finished learned run with fewer than k points inside worst0 < R2: its
// list may miss points beyond worst0, so the query runs again from R2.
template <int D, int K>
__device__ __forceinline__ bool lane_needs_restart(const Lane<D, K>& s, float R2) {
    return uint32_t(s.L[K - 1]) == SENT_IDX && s.w0 < R2;
}

template <int D, int K, bool LEARNED>
__device__ __forceinline__ void lane_finish(const Lane<D, K>& s, const TravArgs& a) {
    if (LEARNED && a.fb_flag) a.fb_flag[s.row] = s.fell_back ? 1 : 0;
    int32_t* oi = a.out_idx + int64_t(s.row) * a.k;
    float* od = a.out_d2 ? a.out_d2 + int64_t(s.row) * a.k : nullptr;
    const int off = K - a.k;
    if (K >= 4 && a.vec_store) {
        // rows are 16-byte aligned: vector stores
#pragma unroll
        for (int j = 0; j < K; j += 4) {
            if (j >= off) {
                int4 vi;
                vi.x = int32_t(uint32_t(s.L[j + 0]));
                vi.y = int32_t(uint32_t(s.L[j + 1]));
                vi.z = int32_t(uint32_t(s.L[j + 2]));
                vi.w = int32_t(uint32_t(s.L[j + 3]));
                float4 vd = make_float4(key_d2(s.L[j]), key_d2(s.L[j + 1]), key_d2(s.L[j + 2]), key_d2(s.L[j + 3]));
                if (vi.x == int32_t(SENT_IDX)) { vi.x = -1; vd.x = __builtin_inff(); }
                if (vi.y == int32_t(SENT_IDX)) { vi.y = -1; vd.y = __builtin_inff(); }
                if (vi.z == int32_t(SENT_IDX)) { vi.z = -1; vd.z = __builtin_inff(); }
                if (vi.w == int32_t(SENT_IDX)) { vi.w = -1; vd.w = __builtin_inff(); }
                *reinterpret_cast<int4*>(oi + (j - off)) = vi;
                if (od) *reinterpret_cast<float4*>(od + (j - off)) = vd;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j >= off) {
                const uint32_t id = uint32_t(s.L[j]);
                const bool empty = id == SENT_IDX;
                oi[j - off] = empty ? -1 : int32_t(id);
                if (od) od[j - off] = empty ? __builtin_inff() : key_d2(s.L[j]);
            }
        }
    }
    if (a.visited) a.visited[s.row] = s.vis;
}

// One loop trip for a lane at node s.curr (record fields c, idx, anc; ids
// is the caller-index array when records hold no index): the state-machine
// step at curr, then up to F fused "return to parent" steps.  Returns the new
// curr (0 = traversal finished).
template <int D, int K, int F, bool CAP = false, bool FAR = true, bool XD = false>
__device__ __forceinline__ int32_t lane_step(Lane<D, K>& s, const float (&c)[D], int32_t idx,
                                             const int32_t* __restrict__ ids,
                                             const float (&anc)[rec_ancestors(D) > 0 ? rec_ancestors(D) : 1],
                                             int32_t N, float cap = 0.0f, int32_t stop = 0,
                                             bool skip = false, uint32_t db = 0) {
    const int32_t curr = s.curr;
    const DimSel<D> dim = split_dim<D, XD, 0>(curr, db);
    float dx[D];
#pragma unroll
    for (int j = 0; j < D; ++j) dx[j] = s.q[j] - c[j];
    const float sd = dim.template rot<0>(dx);
    const bool from_parent = s.prev < curr;
    // skip: the caller found the subtree out of range on entry; it is left
    // at once, as if coming back from it
    const bool enter = from_parent & !skip;
    if (from_parent & skip) ++s.vis;  // entered nodes: this one is left at once
    if (enter) {
        ++s.vis;
        // processNode on the first visit: exact binary32 squared distance,
        // left to right, and insertion into the k-best list
        float d2 = dx[0] * dx[0];
#pragma unroll
        for (int j = 1; j < D; ++j) d2 = d2 + dx[j] * dx[j];
        if constexpr (rec_has_idx(D)) {
            const uint64_t key = make_key(d2, idx);
            if (key < s.L[K - 1]) list_insert<K>(s.L, key);
        } else {
            // the index decides only ties with the worst entry: it is read
            // only when the point can enter the list (d2 <= worst d2)
            if (__float_as_uint(d2) <= uint32_t(s.L[K - 1] >> 32)) {
                const uint64_t key = make_key(d2, ids[curr]);
                if (key < s.L[K - 1]) list_insert<K>(s.L, key);
            }
        }
    }

    // CAP: prune with a tighter bound known to be >= the final k-th distance
    const float worst = CAP ? fminf(key_d2(s.L[K - 1]), cap) : key_d2(s.L[K - 1]);
    const bool far_in = sd * sd <= worst;
    const int32_t close_c = (curr << 1) | (sd > 0.0f ? 1 : 0);
    const int32_t far_c = close_c ^ 1;
    const bool close_missing = close_c > N;
    const bool go_close = enter & !close_missing;
    // the far child is tried when coming from the parent with no close
    // child, or when coming back from the close child (prev == close_c
    // implies prev > curr, i.e. not from the parent)
    const bool try_far = (enter & close_missing) | (s.prev == close_c);
    const bool go_far = try_far & far_in & (far_c <= N);
    bool up = !(go_close | go_far);
    bool far_next = go_far;
    int32_t child = curr;        // node being returned from
    int32_t anc_id = curr >> 1;  // node being returned to
    int32_t next = go_close ? close_c : far_c;
    int32_t nprev = curr;

    // Fused returns.  At ancestor anc_id (depth i above curr: split anc[i],
    // dimension dim-1-i): the lane came from `child`; if that is the close
    // child and the far subtree is in range, step to the far child, else
    // keep returning.
    auto fused = [&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const bool live = up & (anc_id != stop);  // stop: parent of the traversal's root
        {
            if (live) {
                float qa;
                if constexpr (XD) qa = split_dim<D, true, i + 1>(curr, db).template rot<0>(s.q);
                else qa = dim.template rot<i + 1>(s.q);
                const float sda = qa - anc[i];
                const bool child_is_close = (child & 1) == (sda > 0.0f ? 1 : 0);
                const int32_t fa = child ^ 1;
                const bool take_far = child_is_close & (sda * sda <= worst) & (fa <= N);
                if (take_far) {
                    far_next = true;
                    next = fa;
                    nprev = anc_id;
                    up = false;
                } else {
                    child = anc_id;
                    anc_id >>= 1;
                }
            }
        }
    };
    if constexpr (F >= 1) fused(std::integral_constant<int, 0>{});
    if constexpr (F >= 2) fused(std::integral_constant<int, 1>{});
    if constexpr (F >= 3) fused(std::integral_constant<int, 2>{});
    if (up) {
        next = anc_id;  // 0 once the root has returned: finished
        nprev = child;
    }
    s.prev = nprev;
    s.curr = next;
    if (FAR) s.far_entry = far_next;  // read by box tests only
    return next;
}

// Wave-uniform work source.  The Morton-sorted slots are cut into one
// contiguous range per workgroup, so all waves of a workgroup (one CU)
// traverse the same region of the tree and share its L1 working set.
// Workgroups on one XCD (blockIdx % 8) get neighbouring ranges, so the XCD's
// L2 holds one region too.  A wave takes chunks of its group's range until it
// is used up -- chunks shrink as the range drains -- then steals: one lane per
// range reads the cursors of the STEAL_PROBES following ranges (plain atomic
// loads, no read-modify-write), the wave takes the nearest one with enough
// slots left (batched launches: the fullest one) and claims chunks from it
// until it is used up, then looks again.
// Only a range with at least STEAL_MIN slots left is a victim: near the end of
// a balanced batch, moving queries away from the caches that hold their region
// costs more than the idle waves (measured).  Stealing is only a speed-up:
// every range is drained by its own group's waves, so no slot is ever left
// behind.  Cursors sit CURSOR_STRIDE words
// apart so that different ranges' atomics do not share a line.
#ifndef KD_STEAL_PROBES
#define KD_STEAL_PROBES 16
#endif
constexpr uint32_t STEAL_PROBES = KD_STEAL_PROBES;  // at most 64 (one per lane)
#ifndef KD_STEAL_MIN
#define KD_STEAL_MIN 64
#endif
constexpr uint32_t STEAL_MIN = KD_STEAL_MIN;           // single-tree launches: slots a victim must have left
constexpr uint32_t CURSOR_STRIDE = 8;
constexpr uint32_t MAX_GROUPS = 8192;                // persistent workgroups per launch

struct WorkSource {
    uint32_t r0;        // own range
    uint32_t G;         // number of ranges (= workgroups)
    uint32_t src;       // range claimed from: r0 first, then a victim
    uint32_t want;      // next chunk size, 1..64
    uint32_t wpg;       // waves per workgroup
    bool exhausted;
    uint32_t base, extra;  // range r holds base + (r < extra) slots
    uint32_t steal_min;    // slots a victim must have left

    __device__ __forceinline__ WorkSource(uint32_t own, uint32_t groups, uint32_t waves_per_group, uint32_t Q,
                                          uint32_t min_left)
        : r0(own), G(groups), src(own), want(64u), wpg(waves_per_group), exhausted(false), steal_min(min_left) {
        base = Q / G;
        extra = Q - base * G;
    }

    __device__ __forceinline__ uint32_t begin_of(const TravArgs& a, uint32_t r) const {
        (void)a;
        return r * base + (r < extra ? r : extra);
    }

    // FULLEST: victim = the range with most slots left (stealers spread out;
    // costs registers), else the nearest one with at least steal_min left.
    template <bool FULLEST>
    __device__ __forceinline__ void grab(const TravArgs& a, uint32_t lane, uint32_t& cb, uint32_t& cn) {
        cb = 0;
        cn = 0;
        while (!exhausted) {
            const uint32_t r = src;
            const uint32_t beg = begin_of(a, r);
            const uint32_t end = begin_of(a, r + 1);
            uint32_t c = 0;
            if (lane == 0) c = atomicAdd(&a.counter[r * CURSOR_STRIDE], want);
            c = __builtin_amdgcn_readfirstlane(c);
            if (c < end - beg) {
                cb = beg + c;
                cn = end - cb < want ? end - cb : want;
                const uint32_t rem = end - cb - cn;
                const uint32_t w = rem / (2 * wpg);
                want = w < 1 ? 1 : (w > 64 ? 64 : w);
                return;
            }
            // this range is used up: pick the fullest of the following ranges
            const uint32_t probes = G - 1 < STEAL_PROBES ? G - 1 : STEAL_PROBES;
            uint32_t rr = r0 + 1 + lane;
            rr = rr >= G ? rr - G : rr;
            uint32_t left = 0;
            if (lane < probes) {
                const uint32_t size = begin_of(a, rr + 1) - begin_of(a, rr);
                const uint32_t cur =
                    __hip_atomic_load(&a.counter[rr * CURSOR_STRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                left = cur < size ? size - cur : 0;
            }
            // only ranges with a good amount of work left are worth moving
            // queries away from the L1 / L2 that holds their region
            const uint64_t rich = wave_ballot(left >= steal_min);
            if (!rich) {
                exhausted = true;
                return;
            }
            uint32_t best;
            if constexpr (FULLEST) {
                best = left;
#pragma unroll
                for (int m = 32; m >= 1; m >>= 1) {
                    const uint32_t o = __shfl_xor(best, m);
                    best = o > best ? o : best;
                }
                src = __builtin_amdgcn_readlane(rr, int(__builtin_ctzll(wave_ballot(left == best))));
            } else {
                const int at = int(__builtin_ctzll(rich));
                src = __builtin_amdgcn_readlane(rr, at);
                best = __builtin_amdgcn_readlane(left, at);
            }
            const uint32_t w = best / (2 * wpg);
            want = w < 1 ? 1 : (w > 64 ? 64 : w);
        }
    }
};

// Range of workgroup g: groups of one XCD (g % 8) get consecutive ranges.
__device__ __forceinline__ uint32_t group_range(uint32_t g, uint32_t G) {
    if (G % 8 != 0) return g;
    return (g & 7u) * (G >> 3) + (g >> 3);
}

constexpr int max_block(int K) { return K >= 32 ? 256 : 1024; }
// minimum waves per SIMD the register allocation must allow: the 64-entry
// list (128 VGPRs) would otherwise leave room for only two
#ifndef KD_MIN_WAVES_K64
#define KD_MIN_WAVES_K64 3
#endif
constexpr int min_waves(int K) { return K >= 64 ? KD_MIN_WAVES_K64 : 1; }

// Box tests are made only on entering a far child (the side the split-plane
// test lets through most loosely) whose subtree spans at least
// KD_BOX_MIN_HEIGHT levels.

// Idle lanes are refilled once at least refill_min of them are idle: the
// refill's shuffles and list resets run for the whole wave, so waiting for a
// few lanes amortises them at the cost of a few idle lane-trips.  Measured
// (traversal ms, threshold 1 / 4): uniform-1m k = 8 0.689 / 0.698 with the
// paper's rule, 0.679 / 0.654 with subtree boxes; fcp 0.258 / 0.250; k = 64
// (boxes) 7.59 / 7.47; gmm64 k = 8 1.151 / 1.124; clustered-10m k = 16 (boxes)
// 36.0 / 35.7.
#ifndef KD_REFILL_MIN_BATCHED
#define KD_REFILL_MIN_BATCHED 4
#endif

// LDS kernels stage the records of the top tree levels (node ids below
// a.lds_below, at most 64 KB) in the workgroup's LDS at launch; steps at those
// nodes read them from there.  The traversal itself is unchanged.
extern __shared__ uint4 kd_lds_nodes[];

template <int D, int K, int F, bool LEARNED, bool BOX, bool LDSN, bool XD = false>
__global__ __launch_bounds__(max_block(K), min_waves(K)) void knn_persistent(TravArgs a) {
    const TreeRec<D>* __restrict__ g1 = reinterpret_cast<const TreeRec<D>*>(a.nodes);  // indexed by node id
    const int32_t* __restrict__ ids = node_ids<D>(g1, a.N);
    const NodeRec<D>* __restrict__ sq = reinterpret_cast<const NodeRec<D>*>(a.sq);
    TreeRec<D>* lrec = reinterpret_cast<TreeRec<D>*>(kd_lds_nodes);  // indexed by node id
    if constexpr (LDSN) {
        for (int32_t i = int32_t(threadIdx.x) + 1; i < a.lds_below; i += int32_t(blockDim.x)) lrec[i] = g1[i];
        __syncthreads();
    }

    const uint32_t lane = __lane_id();
    const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
    WorkSource ws(group_range(blockIdx.x, gridDim.x), gridDim.x, blockDim.x >> 6, a.Q, STEAL_MIN);
    // Query chunk held across the wave: lane l holds slot cb + l of the
    // current chunk (record and, when learned, initial radius); idle lanes
    // take queries from it by cross-lane shuffle.
    NodeRec<D> chunk;
    float chunk_w0 = 0.0f;
    int32_t chunk_start = 1;
    uint32_t cpos = 0, cn = 0;

    // a lane is active while its curr is a node id (curr = 0: no query; the
    // state machine ends a traversal by stepping to 0)
    Lane<D, K> s;
    s.curr = 0;
    uint32_t restarts = 0;  // learned runs restarted from R2 by this lane
    uint32_t vis_sum = 0;   // entered nodes of this lane's finished and handed-off queries (learned)
    uint32_t wtrip = 0;     // trips of this wave (wave-uniform)
    for (;;) {
        const uint64_t need = wave_ballot(s.curr == 0);
        if (need && !ws.exhausted && uint32_t(__popcll(need)) >= a.refill_min) {
            const uint32_t n = __popcll(need);
            const uint32_t rank = __popcll(need & lt_mask);
            const uint32_t take1 = n < cn - cpos ? n : cn - cpos;
            {
                const int src = int(cpos + (rank < take1 ? rank : 0));
                const NodeRec<D> v = shfl_rec<D>(chunk, src);
                const float vw = LEARNED ? __shfl(chunk_w0, src) : 0.0f;
                const int32_t vs = LEARNED ? __shfl(chunk_start, src) : 1;
                if (s.curr == 0 && rank < take1) {
                    lane_start<D, K, LEARNED>(s, a, v, vw, wtrip, vs);
                }
            }
            cpos += take1;
            if (n > take1) {
                uint32_t cb = 0, cn2 = 0;
                ws.grab<false>(a, lane, cb, cn2);
                if (cn2) {
                    if (lane < cn2) {
                        chunk = load_query<D>(sq + cb + lane);
                        if (LEARNED) {
                            chunk_w0 = a.worst0[cb + lane];
                            chunk_start = a.start[cb + lane];
                        }
                    }
                    cn = cn2;
                    const uint32_t r2 = rank - take1;
                    const uint32_t take2 = n - take1 < cn2 ? n - take1 : cn2;
                    const int src = int(r2 < take2 ? r2 : 0);
                    const NodeRec<D> v = shfl_rec<D>(chunk, src);
                    const float vw = LEARNED ? __shfl(chunk_w0, src) : 0.0f;
                    const int32_t vs = LEARNED ? __shfl(chunk_start, src) : 1;
                    if (s.curr == 0 && rank >= take1 && r2 < take2) {
                        lane_start<D, K, LEARNED>(s, a, v, vw, wtrip, vs);
                    }
                    cpos = take2;
                } else {
                    cn = 0;
                    cpos = 0;
                }
            }
        }
        if (!wave_any(s.curr != 0)) break;
        ++wtrip;
        if (s.curr != 0) {
            float c[D];
            int32_t idx;
            float anc[rec_ancestors(D) > 0 ? rec_ancestors(D) : 1];
            if (LDSN && s.curr < a.lds_below) load_tree<D>(lrec + s.curr, c, idx, anc);
            else load_tree<D>(g1 + s.curr, c, idx, anc);
            const uint32_t db = XD ? uint32_t(a.dims[s.curr]) : 0u;
            bool skip = false;
            if constexpr (BOX) {
                // entering a far subtree of height >= KD_BOX_MIN_HEIGHT:
                // leave it at once when its bounding box is out of range
                if (s.far_entry && s.curr < a.box_below)
                    skip = box_d2<D>(a.boxes, s.curr, s.q) > key_d2(s.L[K - 1]);
            }
            const int32_t stop = LEARNED ? s.stop : 0;
            const int32_t next = lane_step<D, K, F, false, BOX, XD>(s, c, idx, ids, anc, a.N, 0.0f, stop, skip, db);
            const bool done = next == stop;
            bool handed = false;
            // every running lane steps once per wave trip, so a query's trip
            // count is the wave's count since it started; the budget is
            // checked every 16th wave trip (a scalar test), once per query
            if (a.heavy_trips && (wtrip & 15u) == 0 && !done && wtrip - s.t0 - a.heavy_trips < 16u) {
                // over budget: the cooperative kernel finishes this query,
                // unless it already holds heavy_cap queries (then the lane
                // goes on)
                const uint32_t pos = atomicAdd(a.heavy_count, 1u);
                if (pos < a.heavy_cap) {
                    a.heavy_rows[pos] = s.row;
                    if (LEARNED && a.fb_flag) a.fb_flag[s.row] = s.fell_back ? 1 : 2;
                    if (LEARNED) vis_sum += s.vis;
                    s.curr = 0;
                    handed = true;
                }
            }
            if (!handed && done) {
                if (LEARNED && lane_needs_restart<D, K>(s, a.R2)) {
                    s.fell_back = true;
                    ++restarts;
                    lane_reset<D, K>(s, a.k, a.R2);
                } else {
                    if (LEARNED) vis_sum += s.vis;
                    lane_finish<D, K, LEARNED>(s, a);
                    s.curr = 0;  // idle (a learned run may end at its start node's parent)
                }
            }
        }
    }
    if (LEARNED && a.fb_count) {
        // one atomic per wave (all lanes are here: the loop exit is uniform)
        uint64_t vs = vis_sum;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            restarts += __shfl_xor(restarts, m);
            vs += uint64_t(__shfl_xor(uint32_t(vs), m)) | (uint64_t(__shfl_xor(uint32_t(vs >> 32), m)) << 32);
        }
        if (lane == 0 && restarts) atomicAdd(a.fb_count, restarts);
        if (lane == 0 && a.vis_total && vs) atomicAdd(a.vis_total, (unsigned long long)vs);
    }
}

// ------------------------------------------------------------ cooperative
//
// Queries whose traversal exceeds the trip budget (a query far from dense
// data can visit tens of thousands of nodes; one lane would then hold the
// whole launch) are finished here by a whole wave.  The wave walks the top
// levels of the tree with the same state machine, wave-uniformly, processing
// those nodes itself; each node of depth T it steps into is given, with its
// whole subtree, to an idle lane, and the walk goes on as if returning from
// it.  A lane runs the same state machine inside its subtree and stops when
// it steps back out of the subtree root.  The walk and the lanes prune with a
// wave-wide bound that is never below the final k-th distance of the query
// (see coop_bound), so every point of the result is still processed, by
// exactly one lane.  The k best keys of the 64 lists are then merged.  The
// result (indices and squared distances) equals the single-lane traversal's;
// the order and number of processed nodes differ.  Subtrees have about
// 2^KD_COOP_SUB_LEVELS nodes, so a large search spreads over many lanes.
#ifndef KD_COOP_SUB_LEVELS
#define KD_COOP_SUB_LEVELS 9
#endif
// hand-offs are capped at this many rounds of one query per cooperative wave
#ifndef KD_COOP_ROUNDS
#define KD_COOP_ROUNDS 4
#endif
struct CoopArgs {
    const void* nodes;
    const uint8_t* dims;     // stored split dimensions by node id (XD kernel), else NULL
    const float* boxes;      // subtree bounding boxes, or NULL (split planes only)
    int32_t box_below;       // boxes are tested for node ids below this
    int32_t N;
    int T;                   // subtree depth: levels - 1 - KD_COOP_SUB_LEVELS, at least 0
    const float* queries;    // caller [Q][D]
    int k;
    float R2;
    int32_t* out_idx;
    float* out_d2;
    const uint32_t* heavy_count;
    uint32_t heavy_cap;
    const int32_t* heavy_rows;  // [heavy_cap] caller rows; batched: [heavy_cap][2] (job, row)
    const BatchJob* jobs;       // batched hand-off: the tree and outputs come from the job (else NULL)
};

// depth of the cooperative subtrees for a tree of N points
__host__ __device__ __forceinline__ int coop_depth(int32_t N) {
    int levels = 0;
    while (levels < 31 && (int64_t(1) << levels) <= int64_t(N)) ++levels;  // floor(log2 N) + 1
    return levels - 1 - KD_COOP_SUB_LEVELS > 0 ? levels - 1 - KD_COOP_SUB_LEVELS : 0;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t o = __shfl_xor(v, m);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = (uint64_t(uint32_t(__shfl_xor(uint32_t(v >> 32), m))) << 32) |
                           uint32_t(__shfl_xor(uint32_t(v), m));
        v = o < v ? o : v;
    }
    return v;
}

// k-th smallest of the lanes' values (k <= 64), bit by bit from the top:
// bit b of the answer is 0 iff at least k lanes hold a value <= the answer's
// upper bits followed by ones.
__device__ __forceinline__ uint32_t wave_kth_smallest(uint32_t u, int k) {
    uint32_t r = 0;
    for (int b = 31; b >= 0; --b) {
        const uint32_t t = r | ((1u << b) - 1u);
        if (__popcll(wave_ballot(u <= t)) < k) r |= 1u << b;
    }
    return r;
}

// Pruning bound of the cooperative kernel, >= the query's final k-th
// distance: the smaller of (a) the lanes' smallest k-th distance and (b)
// the k-th smallest of the lanes' best distances (k lanes each hold a point
// at most that far).
template <int K>
__device__ __forceinline__ float coop_bound(const uint64_t (&L)[K], int k) {
    uint32_t best = ~0u;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint32_t v = j >= K - k ? uint32_t(L[j] >> 32) : ~0u;
        best = v < best ? v : best;
    }
    const uint32_t a = wave_min_u32(uint32_t(L[K - 1] >> 32));
    const uint32_t b = wave_kth_smallest(best, k);
    return __uint_as_float(a < b ? a : b);
}

template <int D, int K, bool XD = false>
__global__ __launch_bounds__(256) void knn_coop(CoopArgs a) {
    const uint32_t lane = __lane_id();
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    const uint32_t nheavy = *a.heavy_count < a.heavy_cap ? *a.heavy_count : a.heavy_cap;
    for (uint32_t h = wave; h < nheavy; h += nwaves) {
        // the query's tree and outputs: the call's, or (batched) its job's
        const TreeRec<D>* g1;
        const float* boxes;
        const float* queries;
        int32_t box_below, N, k, row;
        int T;
        float R2;
        int32_t* out_idx;
        float* out_d2;
        if (a.jobs) {
            const BatchJob& J = a.jobs[__builtin_amdgcn_readfirstlane(a.heavy_rows[2 * h])];
            row = __builtin_amdgcn_readfirstlane(a.heavy_rows[2 * h + 1]);
            g1 = reinterpret_cast<const TreeRec<D>*>(J.nodes);
            boxes = J.boxes;
            box_below = J.box_below;
            N = J.N;
            T = coop_depth(J.N);
            queries = J.queries;
            k = J.k;
            R2 = J.R2;
            out_idx = J.out_idx;
            out_d2 = J.out_d2;
        } else {
            row = a.heavy_rows[h];
            g1 = reinterpret_cast<const TreeRec<D>*>(a.nodes);
            boxes = a.boxes;
            box_below = a.box_below;
            N = a.N;
            T = a.T;
            queries = a.queries;
            k = a.k;
            R2 = a.R2;
            out_idx = a.out_idx;
            out_d2 = a.out_d2;
        }
        const int32_t* __restrict__ ids = node_ids<D>(g1, N);
        const int32_t first_sub = int32_t(1) << T;  // ids of depth T: [2^T, 2^(T+1))
        Lane<D, K> s;
#pragma unroll
        for (int j = 0; j < D; ++j) s.q[j] = queries[int64_t(row) * D + j];
        s.row = row;
        s.vis = 0;
        lane_reset<D, K>(s, k, R2);
        s.curr = 0;
        int32_t stop = 0;
        // wave-uniform walk of the top levels (the same state machine); a
        // depth-T node it steps into goes to an idle lane as a whole subtree
        int32_t tcurr = 1, tprev = 0;
        bool top_done = false;
        float bound = R2;
        uint32_t trip = 0;
        for (;;) {
            uint64_t idle = wave_ballot(s.curr == 0);
            while (idle && !top_done) {
                if (tcurr == 0) {
                    top_done = true;
                    break;
                }
                if (tcurr >= first_sub) {
                    const uint32_t l = uint32_t(__builtin_ctzll(idle));
                    idle &= idle - 1;
                    if (lane == l) {
                        s.curr = tcurr;
                        s.prev = tcurr >> 1;
                        s.far_entry = true;  // its box is tested on entry
                        stop = tcurr >> 1;
                    }
                    tprev = tcurr;
                    tcurr = tcurr >> 1;
                    continue;
                }
                float c[D];
                int32_t idx;
                load_tree_uniform<D>(g1, tcurr, c, idx);
                const bool from_parent = tprev < tcurr;
                float dx[D];
#pragma unroll
                for (int j = 0; j < D; ++j) dx[j] = s.q[j] - c[j];
                if (from_parent && lane == 0) {
                    float d2 = dx[0] * dx[0];
#pragma unroll
                    for (int j = 1; j < D; ++j) d2 = d2 + dx[j] * dx[j];
                    if (__float_as_uint(d2) <= uint32_t(s.L[K - 1] >> 32)) {
                        const uint64_t key = make_key(d2, rec_has_idx(D) ? idx : ids[tcurr]);
                        if (key < s.L[K - 1]) list_insert<K>(s.L, key);
                    }
                }
                const DimSel<D> dim = split_dim<D, XD, 0>(tcurr, XD ? uint32_t(a.dims[tcurr]) : 0u);
                const float sd = dim.template rot<0>(dx);
                const int32_t close_c = (tcurr << 1) | (sd > 0.0f ? 1 : 0);
                const int32_t far_c = close_c ^ 1;
                const bool far_ok = far_c <= N && sd * sd <= bound;
                int32_t next;
                if (from_parent && close_c <= N) next = close_c;
                else if ((from_parent || tprev == close_c) && far_ok) next = far_c;
                else next = tcurr >> 1;
                tprev = tcurr;
                tcurr = __builtin_amdgcn_readfirstlane(next);
                tprev = __builtin_amdgcn_readfirstlane(tprev);
            }
            if (top_done && !wave_any(s.curr != 0)) break;
            if (s.curr != 0) {
                float c[D];
                int32_t idx;
                float anc[rec_ancestors(D) > 0 ? rec_ancestors(D) : 1];
                load_tree<D>(g1 + s.curr, c, idx, anc);
                const uint32_t db = XD ? uint32_t(a.dims[s.curr]) : 0u;
                const bool skip = boxes != nullptr && s.far_entry && s.curr < box_below &&
                                  box_d2<D>(boxes, s.curr, s.q) > fminf(key_d2(s.L[K - 1]), bound);
                lane_step<D, K, fused_levels(D), true, true, XD>(s, c, idx, ids, anc, N, bound, stop, skip, db);
                if (s.curr == stop) s.curr = 0;
            }
            // the wave-wide bound is refreshed every 8 trips (a stale bound
            // is larger, so still safe to prune with)
            if ((++trip & 7u) == 0) bound = coop_bound<K>(s.L, k);
        }
        // merge: k rounds of the wave-wide smallest key; the lane holding it
        // (keys of points are unique) drops it.  Slots below K - k hold no
        // point: they are set to the largest key first.
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < K - k) s.L[j] = ~uint64_t(0);
        for (int r = 0; r < k; ++r) {
            uint64_t head = s.L[0];
#pragma unroll
            for (int j = 1; j < K; ++j) head = s.L[j] < head ? s.L[j] : head;
            const uint64_t m = wave_min_u64(head);
            const bool empty = uint32_t(m) == SENT_IDX;
            if (lane == 0) {
                out_idx[int64_t(row) * k + r] = empty ? -1 : int32_t(uint32_t(m));
                if (out_d2) out_d2[int64_t(row) * k + r] = empty ? __builtin_inff() : key_d2(m);
            }
            if (!empty && head == m) {
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if (s.L[j] == m) s.L[j] = ~uint64_t(0);
            }
        }
    }
}

__global__ void zero_u32(uint32_t* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}


// lds_bytes > 0: the LDS kernels (plain queries only; the learned kernels
// read every node from global memory)
template <int D, int K>
hipError_t launch_knn(const TravArgs& a, bool learned, int block, int grid, size_t lds_bytes, hipStream_t st) {
    const bool box = a.boxes != nullptr;
    constexpr int F = fused_levels(D);
    const dim3 g(grid), b(block);
    if (a.dims) {
        // stored split dimensions: plain queries, nodes from global memory
        if (learned || lds_bytes) return hipErrorInvalidValue;
        if (box) hipLaunchKernelGGL((knn_persistent<D, K, F, false, true, false, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((knn_persistent<D, K, F, false, false, false, true>), g, b, 0, st, a);
        return hipGetLastError();
    }
    if (learned && box) hipLaunchKernelGGL((knn_persistent<D, K, F, true, true, false>), g, b, 0, st, a);
    else if (learned) hipLaunchKernelGGL((knn_persistent<D, K, F, true, false, false>), g, b, 0, st, a);
    else if (lds_bytes && box) hipLaunchKernelGGL((knn_persistent<D, K, F, false, true, true>), g, b, lds_bytes, st, a);
    else if (lds_bytes) hipLaunchKernelGGL((knn_persistent<D, K, F, false, false, true>), g, b, lds_bytes, st, a);
    else if (box) hipLaunchKernelGGL((knn_persistent<D, K, F, false, true, false>), g, b, 0, st, a);
    else hipLaunchKernelGGL((knn_persistent<D, K, F, false, false, false>), g, b, 0, st, a);
    return hipGetLastError();
}

template <int D>
hipError_t dispatch_k(int K, const TravArgs& a, bool learned, int block, int grid, size_t lds_bytes, hipStream_t st) {
    switch (K) {
        case 1: return launch_knn<D, 1>(a, learned, block, grid, lds_bytes, st);
        case 2: return launch_knn<D, 2>(a, learned, block, grid, lds_bytes, st);
        case 4: return launch_knn<D, 4>(a, learned, block, grid, lds_bytes, st);
        case 8: return launch_knn<D, 8>(a, learned, block, grid, lds_bytes, st);
        case 16: return launch_knn<D, 16>(a, learned, block, grid, lds_bytes, st);
        case 32: return launch_knn<D, 32>(a, learned, block, grid, lds_bytes, st);
        case 64: return launch_knn<D, 64>(a, learned, block, grid, lds_bytes, st);
    }
    return hipErrorInvalidValue;
}

template <int D>
hipError_t occupancy_k(int K, int block, size_t lds_bytes, int* occ) {
    switch (K) {
#define KD_OCC(KK)                                                                                              \
    case KK:                                                                                                    \
        return lds_bytes ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                        \
                               occ, knn_persistent<D, KK, fused_levels(D), false, true, true>, block, lds_bytes) \
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                        \
                               occ, knn_persistent<D, KK, fused_levels(D), true, true, false>, block, 0);
        KD_OCC(1) KD_OCC(2) KD_OCC(4) KD_OCC(8) KD_OCC(16) KD_OCC(32) KD_OCC(64)
#undef KD_OCC
    }
    return hipErrorInvalidValue;
}

hipError_t occupancy(int D, int K, int block, size_t lds_bytes, int* occ) {
    switch (D) {
        case 2: return occupancy_k<2>(K, block, lds_bytes, occ);
        case 3: return occupancy_k<3>(K, block, lds_bytes, occ);
        case 4: return occupancy_k<4>(K, block, lds_bytes, occ);
    }
    return hipErrorInvalidValue;
}

hipError_t dispatch_dk(int D, int K, const TravArgs& a, bool learned, int block, int grid, size_t lds_bytes,
                       hipStream_t st) {
    switch (D) {
        case 2: return dispatch_k<2>(K, a, learned, block, grid, lds_bytes, st);
        case 3: return dispatch_k<3>(K, a, learned, block, grid, lds_bytes, st);
        case 4: return dispatch_k<4>(K, a, learned, block, grid, lds_bytes, st);
    }
    return hipErrorInvalidValue;
}

template <int D>
hipError_t launch_coop_k(int K, const CoopArgs& a, int grid, hipStream_t st) {
    const dim3 g(grid), b(256);
    if (a.dims) {
        if (a.jobs) return hipErrorInvalidValue;  // batches hold level-rule trees only
        switch (K) {
            case 1: hipLaunchKernelGGL((knn_coop<D, 1, true>), g, b, 0, st, a); break;
            case 2: hipLaunchKernelGGL((knn_coop<D, 2, true>), g, b, 0, st, a); break;
            case 4: hipLaunchKernelGGL((knn_coop<D, 4, true>), g, b, 0, st, a); break;
            case 8: hipLaunchKernelGGL((knn_coop<D, 8, true>), g, b, 0, st, a); break;
            case 16: hipLaunchKernelGGL((knn_coop<D, 16, true>), g, b, 0, st, a); break;
            case 32: hipLaunchKernelGGL((knn_coop<D, 32, true>), g, b, 0, st, a); break;
            case 64: hipLaunchKernelGGL((knn_coop<D, 64, true>), g, b, 0, st, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (K) {
        case 1: hipLaunchKernelGGL((knn_coop<D, 1>), g, b, 0, st, a); break;
        case 2: hipLaunchKernelGGL((knn_coop<D, 2>), g, b, 0, st, a); break;
        case 4: hipLaunchKernelGGL((knn_coop<D, 4>), g, b, 0, st, a); break;
        case 8: hipLaunchKernelGGL((knn_coop<D, 8>), g, b, 0, st, a); break;
        case 16: hipLaunchKernelGGL((knn_coop<D, 16>), g, b, 0, st, a); break;
        case 32: hipLaunchKernelGGL((knn_coop<D, 32>), g, b, 0, st, a); break;
        case 64: hipLaunchKernelGGL((knn_coop<D, 64>), g, b, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_coop(int D, int K, const CoopArgs& a, int grid, hipStream_t st) {
    switch (D) {
        case 2: return launch_coop_k<2>(K, a, grid, st);
        case 3: return launch_coop_k<3>(K, a, grid, st);
        case 4: return launch_coop_k<4>(K, a, grid, st);
    }
    return hipErrorInvalidValue;
}

size_t rec_bytes(int D) {
    switch (D) {
        case 2: return sizeof(NodeRec<2>);
        case 3: return sizeof(NodeRec<3>);
        default: return sizeof(NodeRec<4>);
    }
}

// ------------------------------------------------------------ batched jobs
//
// Many trees in one launch: the jobs of one (dimension, K) class share a
// class slot space (jobs back to back, each job's queries Morton-sorted).  A
// lane carries its job's tree pointer, size, k and output pointers along with
// the query, so the lanes of one wave may serve different trees; the state
// machine is the same code as the single-tree kernel.

// Class query record: coordinates, caller row, job index (32 bytes).
struct alignas(32) BRec {
    float c[4];
    int32_t row;
    int32_t job;
    int32_t pad[2];
};

template <int D>
__global__ void batch_gather(const BatchJob* __restrict__ jobs, int njobs, const uint32_t* __restrict__ perm,
                             uint32_t n, BRec* __restrict__ recs) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t slot = perm ? perm[i] : i;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].slot_base <= slot) lo = mid;
        else hi = mid - 1;
    }
    const BatchJob& J = jobs[lo];
    const uint32_t row = slot - J.slot_base;
    BRec r;
#pragma unroll
    for (int d = 0; d < 4; ++d) r.c[d] = d < D ? J.queries[size_t(row) * D + d] : 0.0f;
    r.row = int32_t(row);
    r.job = lo;
    r.pad[0] = r.pad[1] = 0;
    recs[i] = r;
}

struct BatchArgs {
    const BatchJob* jobs;
    const BRec* recs;
    uint32_t Q;
    uint32_t* counter;
    const float* worst0;     // learned kernels: initial squared radius per record (jobs with a model)
    uint32_t heavy_trips;    // trip budget per query before the hand-off, 0 = none
    uint32_t heavy_cap;
    uint32_t* heavy_count;
    int32_t* heavy_rows;     // [heavy_cap][2]: (job, row)
};

template <int D, int K>
struct JobLane {
    const TreeRec<D>* g1;  // the lane's tree, indexed by node id
    const float* boxes;    // its subtree bounding boxes (NULL: split planes only)
    int32_t box_below;
    const int32_t* ids;    // its caller-index array (records without index)
    int32_t N;
    int32_t k;
    int32_t* oi;
    float* od;
    int32_t vec;
    int32_t job;
    float R2;
};

template <int D, int K, bool LEARNED = false>
__device__ __forceinline__ void batch_start(Lane<D, K>& s, JobLane<D, K>& j, const BatchJob* jobs,
                                            const BRec& r, float w0 = 0.0f, uint32_t wtrip = 0) {
    const BatchJob& J = jobs[r.job];
    j.job = r.job;
    j.R2 = J.R2;
    j.g1 = reinterpret_cast<const TreeRec<D>*>(J.nodes);
    j.boxes = J.boxes;
    j.box_below = J.box_below;
    j.ids = node_ids<D>(j.g1, J.N);
    j.N = J.N;
    j.k = J.k;
    j.oi = J.out_idx;
    j.od = J.out_d2;
    j.vec = J.vec_store;
#pragma unroll
    for (int d = 0; d < D; ++d) s.q[d] = r.c[d];
    s.row = r.row;
    s.vis = 0;
    s.t0 = wtrip;
    s.fell_back = false;
    // learned: jobs with a model start from their initial radius
    lane_reset<D, K>(s, j.k, LEARNED && J.learned ? w0 : J.R2);
}

template <int D, int K>
__device__ __forceinline__ void batch_finish(const Lane<D, K>& s, const JobLane<D, K>& j) {
    int32_t* oi = j.oi + int64_t(s.row) * j.k;
    float* od = j.od ? j.od + int64_t(s.row) * j.k : nullptr;
    const int off = K - j.k;
#pragma unroll
    for (int e = 0; e < K; ++e) {
        if (e >= off) {
            const uint32_t id = uint32_t(s.L[e]);
            const bool empty = id == SENT_IDX;
            oi[e - off] = empty ? -1 : int32_t(id);
            if (od) od[e - off] = empty ? __builtin_inff() : key_d2(s.L[e]);
        }
    }
}

__device__ __forceinline__ BRec shfl_brec(const BRec& r, int src) {
    BRec o;
#pragma unroll
    for (int d = 0; d < 4; ++d) o.c[d] = __shfl(r.c[d], src);
    o.row = __shfl(r.row, src);
    o.job = __shfl(r.job, src);
    o.pad[0] = o.pad[1] = 0;
    return o;
}

__device__ __forceinline__ BRec load_brec(const BRec* p) {
    const float4 a = reinterpret_cast<const float4*>(p)[0];
    const int4 b = reinterpret_cast<const int4*>(p)[1];
    BRec r;
    r.c[0] = a.x;
    r.c[1] = a.y;
    r.c[2] = a.z;
    r.c[3] = a.w;
    r.row = b.x;
    r.job = b.y;
    r.pad[0] = r.pad[1] = 0;
    return r;
}

template <int D, int K, int F, bool LEARNED>
__global__ __launch_bounds__(max_block(K)) void knn_batched(BatchArgs a) {
    const uint32_t lane = __lane_id();
    const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
    // the work source only reads a.Q and a.counter
    TravArgs wa = {};
    wa.Q = a.Q;
    wa.counter = a.counter;
    // the classes of a batch mix trees and k, so their ranges drain unevenly:
    // any slot left is worth stealing
    WorkSource ws(group_range(blockIdx.x, gridDim.x), gridDim.x, blockDim.x >> 6, a.Q, 1u);
    BRec chunk;
    float chunk_w0 = 0.0f;
    uint32_t cpos = 0, cn = 0;
    Lane<D, K> s;
    s.curr = 0;  // active while curr != 0, as in the single-tree kernel
    JobLane<D, K> j;
    uint32_t wtrip = 0;  // trips of this wave (wave-uniform)
    for (;;) {
        const uint64_t need = wave_ballot(s.curr == 0);
        if (need && !ws.exhausted && __popcll(need) >= KD_REFILL_MIN_BATCHED) {
            const uint32_t n = __popcll(need);
            const uint32_t rank = __popcll(need & lt_mask);
            const uint32_t take1 = n < cn - cpos ? n : cn - cpos;
            {
                const int src = int(cpos + (rank < take1 ? rank : 0));
                const BRec v = shfl_brec(chunk, src);
                const float vw = LEARNED ? __shfl(chunk_w0, src) : 0.0f;
                if (s.curr == 0 && rank < take1) {
                    batch_start<D, K, LEARNED>(s, j, a.jobs, v, vw, wtrip);
                }
            }
            cpos += take1;
            if (n > take1) {
                uint32_t cb = 0, cn2 = 0;
                ws.grab<true>(wa, lane, cb, cn2);
                if (cn2) {
                    if (lane < cn2) {
                        chunk = load_brec(a.recs + cb + lane);
                        if (LEARNED) chunk_w0 = a.worst0[cb + lane];
                    }
                    cn = cn2;
                    const uint32_t r2 = rank - take1;
                    const uint32_t take2 = n - take1 < cn2 ? n - take1 : cn2;
                    const int src = int(r2 < take2 ? r2 : 0);
                    const BRec v = shfl_brec(chunk, src);
                    const float vw = LEARNED ? __shfl(chunk_w0, src) : 0.0f;
                    if (s.curr == 0 && rank >= take1 && r2 < take2) {
                        batch_start<D, K, LEARNED>(s, j, a.jobs, v, vw, wtrip);
                    }
                    cpos = take2;
                } else {
                    cn = 0;
                    cpos = 0;
                }
            }
        }
        if (!wave_any(s.curr != 0)) break;
        ++wtrip;
        if (s.curr != 0) {
            float c[D];
            int32_t idx;
            float anc[rec_ancestors(D) > 0 ? rec_ancestors(D) : 1];
            load_tree<D>(j.g1 + s.curr, c, idx, anc);
            // subtree box test as in knn_persistent (jobs may mix rules)
            const bool skip = s.far_entry && s.curr < j.box_below && j.boxes != nullptr &&
                              box_d2<D>(j.boxes, s.curr, s.q) > key_d2(s.L[K - 1]);
            const int32_t next = lane_step<D, K, F>(s, c, idx, j.ids, anc, j.N, 0.0f, 0, skip);
            bool handed = false;
            // over the trip budget (checked every 16th wave trip, once per
            // query): the cooperative kernel finishes the query from R2
            if (a.heavy_trips && (wtrip & 15u) == 0 && next != 0 && wtrip - s.t0 - a.heavy_trips < 16u) {
                const uint32_t pos = atomicAdd(a.heavy_count, 1u);
                if (pos < a.heavy_cap) {
                    a.heavy_rows[2 * pos] = j.job;
                    a.heavy_rows[2 * pos + 1] = s.row;
                    s.curr = 0;
                    handed = true;
                }
            }
            if (!handed && next == 0) {
                if (LEARNED && lane_needs_restart<D, K>(s, j.R2)) {
                    // fewer than k points inside the initial radius: again from R2
                    s.fell_back = true;
                    lane_reset<D, K>(s, j.k, j.R2);
                } else {
                    batch_finish<D, K>(s, j);
                }
            }
        }
    }
}

template <int D, int K>
hipError_t launch_batched(const BatchArgs& a, int block, int grid, hipStream_t st) {
    // learned-radius kernels exist for 3-D jobs only (the model is 3-D)
    if constexpr (D == 3) {
        if (a.worst0) {
            hipLaunchKernelGGL((knn_batched<D, K, fused_levels(D), true>), dim3(grid), dim3(block), 0, st, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((knn_batched<D, K, fused_levels(D), false>), dim3(grid), dim3(block), 0, st, a);
    return hipGetLastError();
}

template <int D>
hipError_t dispatch_batched_k(int K, const BatchArgs& a, int block, int grid, hipStream_t st) {
    switch (K) {
        case 1: return launch_batched<D, 1>(a, block, grid, st);
        case 2: return launch_batched<D, 2>(a, block, grid, st);
        case 4: return launch_batched<D, 4>(a, block, grid, st);
        case 8: return launch_batched<D, 8>(a, block, grid, st);
        case 16: return launch_batched<D, 16>(a, block, grid, st);
        case 32: return launch_batched<D, 32>(a, block, grid, st);
        case 64: return launch_batched<D, 64>(a, block, grid, st);
    }
    return hipErrorInvalidValue;
}

template <int D>
hipError_t occupancy_batched_k(int K, int block, int* occ) {
    switch (K) {
#define KD_OCCB(KK) case KK: return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, knn_batched<D, KK, fused_levels(D), D == 3>, block, 0);
        KD_OCCB(1) KD_OCCB(2) KD_OCCB(4) KD_OCCB(8) KD_OCCB(16) KD_OCCB(32) KD_OCCB(64)
#undef KD_OCCB
    }
    return hipErrorInvalidValue;
}

// worst0[slot] = min(R2, fl(r0 * r0)) for r0 = r0_rows[row of slot]; a
// non-finite or negative r0 gives R2 (the learned-radius rule).
template <int D>
__global__ void radius_to_worst0(const float* __restrict__ r0_rows, const NodeRec<D>* __restrict__ sq, uint32_t Q,
                                 float R2, float* __restrict__ worst0) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q) return;
    const float r0 = r0_rows[sq[i].idx];
    float w = R2;
    if (__builtin_isfinite(r0) && r0 >= 0.0f) {
        const float r2 = r0 * r0;
        w = r2 < R2 ? r2 : R2;
    }
    worst0[i] = w;
}

// Start node of a learned initial-radius run.  Descending from the root, a
// node whose split plane lies farther from the query than the initial radius
// (fl(sd * sd) > worst0, strictly) has its own point and every point of its
// far subtree farther than worst0 too: such a point p has d2 >= fl(sd * sd)
// (rounding is monotone and d2 sums non-negative squares).  Only the close
// child's subtree can then hold points within worst0, so the run may start at
// the deepest node reached this way; a run that finds fewer than k points
// within worst0 there restarts from the root at R2 as before.  At most
// floor(log2 N) + 1 steps (ids double; N < 2^30).
template <int D>
__global__ void learned_start(const TreeRec<D>* __restrict__ g1, int32_t N, const NodeRec<D>* __restrict__ sq,
                              const float* __restrict__ worst0, uint32_t Q, int32_t* __restrict__ start) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q) return;
    const NodeRec<D> r = sq[i];
    const float w0 = worst0[i];
    int32_t curr = 1;
    for (;;) {
        float c[D];
        int32_t idx;
        float anc[rec_ancestors(D) > 0 ? rec_ancestors(D) : 1];
        load_tree<D>(g1 + curr, c, idx, anc);
        const DimSel<D> dim(curr);
        float dx[D];
#pragma unroll
        for (int j = 0; j < D; ++j) dx[j] = r.c[j] - c[j];
        const float sd = dim.template rot<0>(dx);
        if (!(sd * sd > w0)) break;
        const int32_t cc = (curr << 1) | (sd > 0.0f ? 1 : 0);
        if (cc > N) break;
        curr = cc;
    }
    start[i] = curr;
}

hipError_t launch_learned_start(int D, const void* nodes, int32_t N, const void* sq, const float* worst0, uint32_t Q,
                                int32_t* start, hipStream_t st) {
    if (Q == 0) return hipSuccess;
    const dim3 grid((Q + 255) / 256), block(256);
    switch (D) {
        case 2: hipLaunchKernelGGL(learned_start<2>, grid, block, 0, st, (const TreeRec<2>*)nodes, N,
                                   (const NodeRec<2>*)sq, worst0, Q, start); break;
        case 3: hipLaunchKernelGGL(learned_start<3>, grid, block, 0, st, (const TreeRec<3>*)nodes, N,
                                   (const NodeRec<3>*)sq, worst0, Q, start); break;
        default: hipLaunchKernelGGL(learned_start<4>, grid, block, 0, st, (const TreeRec<4>*)nodes, N,
                                    (const NodeRec<4>*)sq, worst0, Q, start); break;
    }
    return hipGetLastError();
}

hipError_t launch_radius_to_worst0(int D, const float* r0, const void* sq, uint32_t Q, float R2, float* worst0,
                                   hipStream_t st) {
    const dim3 grid((Q + 255) / 256), block(256);
    switch (D) {
        case 2: hipLaunchKernelGGL(radius_to_worst0<2>, grid, block, 0, st, r0, (const NodeRec<2>*)sq, Q, R2, worst0); break;
        case 3: hipLaunchKernelGGL(radius_to_worst0<3>, grid, block, 0, st, r0, (const NodeRec<3>*)sq, Q, R2, worst0); break;
        default: hipLaunchKernelGGL(radius_to_worst0<4>, grid, block, 0, st, r0, (const NodeRec<4>*)sq, Q, R2, worst0); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t batch_rec_bytes() { return sizeof(BRec); }
// hand-off count (one cache line), then the range cursors
size_t batch_cursor_bytes() { return 256 + size_t(MAX_GROUPS) * CURSOR_STRIDE * 4; }
uint32_t batch_heavy_cap(int device) { return uint32_t(device_info(device).cus) * 2u * 4u * KD_COOP_ROUNDS; }

// One (dim, K) class of a batched call: gather into class records, initial
// radii of the jobs with a model, zero the counters, one persistent traversal
// launch, then the cooperative kernel for queries over the trip budget.
kd_status run_batch_class(const BatchJob* d_jobs, int njobs, int dim, int K, uint32_t n, const uint32_t* perm,
                          void* recs, uint32_t* counters, const QueryPlan& plan, int device, hipStream_t st,
                          const BatchLearned* learned, int32_t* heavy_rows) {
    if (n == 0) return KD_OK;
    const DeviceInfo& dev = device_info(device);
    const dim3 g((n + 255) / 256), b(256);
    switch (dim) {
        case 2: hipLaunchKernelGGL(batch_gather<2>, g, b, 0, st, d_jobs, njobs, perm, n, (BRec*)recs); break;
        case 3: hipLaunchKernelGGL(batch_gather<3>, g, b, 0, st, d_jobs, njobs, perm, n, (BRec*)recs); break;
        default: hipLaunchKernelGGL(batch_gather<4>, g, b, 0, st, d_jobs, njobs, perm, n, (BRec*)recs); break;
    }
    KD_HIP(hipGetLastError());
    float* worst0 = nullptr;
    if (learned && dim == 3) {
        worst0 = learned->worst0;
        KD_HIP(launch_mlp_worst0_jobs(learned->jobs, learned->njobs, learned->ntiles, recs, worst0, st));
    }
    int block = plan.block;
    if (K >= 32 && block > 256) block = 256;
    int occ = 0;
    hipError_t e = dim == 2 ? occupancy_batched_k<2>(K, block, &occ)
                 : dim == 3 ? occupancy_batched_k<3>(K, block, &occ) : occupancy_batched_k<4>(K, block, &occ);
    if (e != hipSuccess) return hip_error(e, "occupancy query");
    int64_t per_cu = plan.waves_per_cu / (block / 64);
    if (per_cu < 1) per_cu = 1;
    if (occ > 0 && per_cu > occ) per_cu = occ;
    int64_t grid = int64_t(dev.cus) * per_cu;
    const int64_t need = (int64_t(n) + block - 1) / block;
    if (grid > need) grid = need;
    if (grid > MAX_GROUPS) grid = MAX_GROUPS;
    if (grid > 8 && grid % 8) grid -= grid % 8;
    if (grid < 1) grid = 1;
    // counters: hand-off count at word 0, range cursors from word 64
    const int nzero = 64 + int(grid) * int(CURSOR_STRIDE);
    hipLaunchKernelGGL(zero_u32, dim3(unsigned((nzero + 255) / 256)), dim3(256), 0, st, counters, nzero);
    KD_HIP(hipGetLastError());
    const bool use_boxes = plan.prune != 1;
    const int heavy_trips = plan.heavy_default ? (use_boxes ? KD_DEFAULT_HEAVY_TRIPS_BOXES : KD_DEFAULT_HEAVY_TRIPS)
                                               : plan.heavy_trips;
    BatchArgs a = {};
    a.jobs = d_jobs;
    a.recs = reinterpret_cast<const BRec*>(recs);
    a.Q = n;
    a.counter = counters + 64;
    a.worst0 = worst0;
    if (heavy_trips > 0 && heavy_rows) {
        a.heavy_trips = uint32_t(heavy_trips);
        a.heavy_cap = batch_heavy_cap(device);
        a.heavy_count = counters;
        a.heavy_rows = heavy_rows;
    }
    e = dim == 2 ? dispatch_batched_k<2>(K, a, block, int(grid), st)
      : dim == 3 ? dispatch_batched_k<3>(K, a, block, int(grid), st) : dispatch_batched_k<4>(K, a, block, int(grid), st);
    if (e != hipSuccess) return hip_error(e, "knn_batched launch");
    if (a.heavy_trips) {
        // handed-off queries, one wave each; the count is read on the device
        CoopArgs c = {};
        c.heavy_count = a.heavy_count;
        c.heavy_cap = a.heavy_cap;
        c.heavy_rows = heavy_rows;
        c.jobs = d_jobs;
        e = launch_coop(dim, K, c, dev.cus * 2, st);
        if (e != hipSuccess) return hip_error(e, "knn_coop launch (batched)");
    }
    return KD_OK;
}

int k_template(int k) {
    int K = 1;
    while (K < k) K <<= 1;
    return K;
}

// Per-stream scratch of one query call, laid out as run_knn uses it:
// [range cursors | restart count | hand-off count] (256 KB + 4 KB), traversal
// records, sort ping-pong buffers and histograms, initial radii (learned),
// hand-off rows.
size_t query_scratch_bytes(int64_t Q, int dim, bool sorted, bool learned, bool handoff) {
    const size_t cursor_bytes = size_t(MAX_GROUPS) * CURSOR_STRIDE * 4;
    const size_t head = cursor_bytes + 4096;
    const size_t sq_bytes = (size_t(Q) * rec_bytes(dim) + 255) & ~size_t(255);
    const size_t sort_bytes = sorted ? sort_scratch_bytes(Q, dim) : 0;
    const size_t q4 = (size_t(Q) * 4 + 255) & ~size_t(255);
    return head + sq_bytes + sort_bytes + (learned ? 2 * q4 : 0) + (handoff ? q4 : 0);
}

namespace {
// Five events bracketing the stages of one query call (sort, initial radius,
// traversal, hand-off), destroyed with the call.
struct StageEvents {
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    kd_status create() {
        for (auto& e : ev) KD_HIP(hipEventCreate(&e));
        return KD_OK;
    }
    ~StageEvents() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};
}  // namespace

kd_status run_knn(kd_tree t, const float* queries, int64_t Q, const QueryPlan& plan, int32_t* out_idx,
                  float* out_d2, uint32_t* visited, kd_stream stream, const LearnedSpec* learned,
                  kd_stats* stats, const FixedScratch* fixed) {
    if (t->d_dims && (learned || plan.lds_levels > 0))
        return set_error(KD_EUNSUPPORTED, "trees with stored split dimensions take plain queries with nodes read "
                                          "from global memory (no learned radius, opts.lds_levels 0)");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const DeviceInfo& dev = device_info(t->device);
    void* ws = nullptr;
    // scratch: [range cursors | restart count | hand-off count] queries  sort
    //          worst0  hand-off rows
    // The per-query visited count is the single-lane traversal's, so there
    // is no hand-off when it is requested.
    // subtree boxes unless the paper's rule is asked for, explicitly or by
    // requesting its processed-node count
    const bool use_boxes = plan.prune == 2 || (plan.prune == 0 && visited == nullptr);
    // trip budget: boxes shorten the long traversals, so their default is
    // longer (gmm64-1m k = 8: 1.53 ms at 1024, 1.33 ms at 4096)
    const int heavy_trips = plan.heavy_default && use_boxes ? KD_DEFAULT_HEAVY_TRIPS_BOXES : plan.heavy_trips;
    const bool handoff = heavy_trips > 0 && visited == nullptr;
    const size_t cursor_bytes = size_t(MAX_GROUPS) * CURSOR_STRIDE * 4;  // 256 KB
    const size_t head = cursor_bytes + 4096;
    const size_t sq_bytes = (size_t(Q) * rec_bytes(t->dim) + 255) & ~size_t(255);
    const size_t sort_bytes = plan.sort_bits > 0 ? sort_scratch_bytes(Q, t->dim) : 0;
    const size_t q4 = (size_t(Q) * 4 + 255) & ~size_t(255);
    const size_t learn_bytes = learned ? 2 * q4 : 0;  // initial radii, start nodes
    const size_t ws_bytes = query_scratch_bytes(Q, t->dim, plan.sort_bits > 0, learned != nullptr, handoff);
    kd_status s = KD_OK;
    if (fixed) {
        if (ws_bytes > fixed->bytes)
            return set_error(KD_EINVAL, "query scratch of " + std::to_string(ws_bytes) +
                                            " bytes exceeds the fixed scratch of " + std::to_string(fixed->bytes) +
                                            " bytes (too many queries for this entry point)");
        ws = fixed->ptr;
    } else {
        s = scratch(stream, ws_bytes, &ws);
        if (s != KD_OK) return s;
    }
    // timing events only for calls that may create them
    auto tbegin = [&](hipEvent_t* ev) -> kd_status {
        *ev = nullptr;
        return fixed ? KD_OK : timing_begin(st, ev);
    };
    char* base = static_cast<char*>(ws);
    uint32_t* counter1 = reinterpret_cast<uint32_t*>(base);
    uint32_t* fb_count = reinterpret_cast<uint32_t*>(base + cursor_bytes);
    uint32_t* heavy_count = reinterpret_cast<uint32_t*>(base + cursor_bytes + 4);
    unsigned long long* vis_total = reinterpret_cast<unsigned long long*>(base + cursor_bytes + 8);
    void* sq = base + head;
    void* sort_ws = base + head + sq_bytes;
    float* worst0 = learned ? reinterpret_cast<float*>(base + head + sq_bytes + sort_bytes) : nullptr;
    int32_t* start = learned ? reinterpret_cast<int32_t*>(base + head + sq_bytes + sort_bytes + q4) : nullptr;
    int32_t* heavy_rows = handoff ? reinterpret_cast<int32_t*>(base + head + sq_bytes + sort_bytes + learn_bytes)
                                  : nullptr;
    // range cursors, restart count, hand-off count, entered-node total (64-bit)
    const uint32_t n_counters = uint32_t(cursor_bytes / 4) + 4;

    // stage events for the caller's stats (stage times need a synchronisation,
    // which stats implies)
    StageEvents sev;
    if (stats) {
        s = sev.create();
        if (s != KD_OK) return s;
        KD_HIP(hipEventRecord(sev.ev[0], st));
    }

    // query reorder: Morton sort whose last pass writes the traversal records
    hipEvent_t evs;
    s = tbegin(&evs);
    if (s != KD_OK) return s;
    hipError_t e = hipSuccess;
    s = reorder_queries(t, queries, Q, plan.sort_bits, sort_ws, sq, counter1, n_counters, st);
    if (s != KD_OK) return s;
    s = timing_end(st, evs, "sort");
    if (s != KD_OK) return s;
    if (stats) KD_HIP(hipEventRecord(sev.ev[1], st));

    if (learned) {
        hipEvent_t evm;
        s = tbegin(&evm);
        if (s != KD_OK) return s;
        if (learned->params)
            e = launch_mlp_worst0(learned->params, learned->lo, learned->inv, learned->margin, plan.R2, sq,
                                  uint32_t(Q), worst0, st);
        else
            e = launch_radius_to_worst0(t->dim, learned->r0, sq, uint32_t(Q), plan.R2, worst0, st);
        if (e != hipSuccess) return hip_error(e, "initial radius launch");
        e = launch_learned_start(t->dim, t->d_nodes, int32_t(t->N), sq, worst0, uint32_t(Q), start, st);
        if (e != hipSuccess) return hip_error(e, "start node launch");
        s = timing_end(st, evm, "mlp");
        if (s != KD_OK) return s;
    }
    if (stats) KD_HIP(hipEventRecord(sev.ev[2], st));

    TravArgs a = {};
    a.nodes = t->d_nodes;
    a.dims = t->d_dims;
    a.boxes = use_boxes ? static_cast<const float*>(t->d_boxes) : nullptr;
    a.box_below = box_id_limit(t->N);
    a.refill_min = (use_boxes || plan.K == 1) ? 4u : 1u;  // measured best, see KD_REFILL_MIN_BATCHED
    // top levels in LDS (plain queries): ids 1 .. min(2^L, N + 1) - 1
    size_t lds_bytes = 0;
    if (plan.lds_levels > 0 && !learned) {
        const int64_t below = std::min<int64_t>(int64_t(1) << plan.lds_levels, t->N + 1);
        a.lds_below = int32_t(below);
        lds_bytes = size_t(below) * 4 * size_t(rec_words(t->dim));
    }
    a.N = int32_t(t->N);
    a.sq = sq;
    a.Q = uint32_t(Q);
    a.k = plan.k;
    a.R2 = plan.R2;
    a.out_idx = out_idx;
    a.out_d2 = out_d2;
    a.visited = visited;
    a.counter = counter1;
    a.vec_store = (plan.k % 4 == 0) && (reinterpret_cast<uintptr_t>(out_idx) % 16 == 0) &&
                  (reinterpret_cast<uintptr_t>(out_d2) % 16 == 0);
    if (learned) {
        a.worst0 = worst0;
        a.start = start;
        a.fb_count = fb_count;
        a.fb_flag = learned->fb_flag;
        a.vis_total = vis_total;
    }
    const int coop_grid = dev.cus * 2;                      // workgroups of 4 waves
    const uint32_t heavy_cap = uint32_t(coop_grid) * 4u * KD_COOP_ROUNDS;  // rounds of one query per wave
    if (handoff) {
        a.heavy_trips = uint32_t(heavy_trips);
        a.heavy_cap = heavy_cap;
        a.heavy_count = heavy_count;
        a.heavy_rows = heavy_rows;
    }

    int block = plan.block;
    if (plan.K >= 32 && block > 256) block = 256;
    const int waves_per_block = block / 64;
    int occ = 0;
    e = occupancy(t->dim, plan.K, block, lds_bytes, &occ);
    if (e != hipSuccess) return hip_error(e, "occupancy query");
    int64_t per_cu = plan.waves_per_cu / waves_per_block;
    if (per_cu < 1) per_cu = 1;
    if (occ > 0 && per_cu > occ) per_cu = occ;  // one round of resident workgroups
    int64_t grid = int64_t(dev.cus) * per_cu;
    const int64_t need = (Q + block - 1) / block;
    if (grid > need) grid = need;
    if (grid > MAX_GROUPS) grid = MAX_GROUPS;
    if (grid > 8 && grid % 8) grid -= grid % 8;
    if (grid < 1) grid = 1;
    hipEvent_t ev0;
    s = tbegin(&ev0);
    if (s != KD_OK) return s;
    e = dispatch_dk(t->dim, plan.K, a, learned != nullptr, block, int(grid), lds_bytes, st);
    if (e != hipSuccess) return hip_error(e, "knn_persistent launch");
    s = timing_end(st, ev0, "traverse");
    if (s != KD_OK) return s;
    if (stats) KD_HIP(hipEventRecord(sev.ev[3], st));
    if (handoff) {
        // queries over the trip budget, one wave each (the count is read on
        // the device; waves beyond it exit at once)
        CoopArgs c = {};
        c.nodes = t->d_nodes;
        c.dims = t->d_dims;
        c.boxes = a.boxes;
        c.box_below = a.box_below;
        c.N = int32_t(t->N);
        c.T = coop_depth(int32_t(t->N));
        c.queries = queries;
        c.k = plan.k;
        c.R2 = plan.R2;
        c.out_idx = out_idx;
        c.out_d2 = out_d2;
        c.heavy_count = heavy_count;
        c.heavy_cap = heavy_cap;
        c.heavy_rows = heavy_rows;
        hipEvent_t evc;
        s = tbegin(&evc);
        if (s != KD_OK) return s;
        e = launch_coop(t->dim, plan.K, c, coop_grid, st);
        if (e != hipSuccess) return hip_error(e, "knn_coop launch");
        s = timing_end(st, evc, "coop");
        if (s != KD_OK) return s;
    }
    if (stats) {
        KD_HIP(hipEventRecord(sev.ev[4], st));
        uint32_t cnt[4] = {0, 0, 0, 0};  // restarts, hand-offs, entered nodes (lo, hi)
        KD_HIP(hipMemcpyAsync(cnt, fb_count, sizeof(cnt), hipMemcpyDeviceToHost, st));
        KD_HIP(hipStreamSynchronize(st));
        stats->queries = Q;
        stats->fallbacks = cnt[0];
        stats->handed_off = handoff ? std::min(cnt[1], heavy_cap) : 0;
        stats->visited = learned ? int64_t(uint64_t(cnt[2]) | (uint64_t(cnt[3]) << 32)) : -1;
        float* ms[4] = {&stats->sort_ms, &stats->radius_ms, &stats->traverse_ms, &stats->handoff_ms};
        for (int i = 0; i < 4; ++i) KD_HIP(hipEventElapsedTime(ms[i], sev.ev[i], sev.ev[i + 1]));
    }
    return KD_OK;
}

// ------------------------------------------------------------ range queries
//
// All points within a radius of a query, or inside an axis-aligned box: the
// un-ordered form of the same state machine (Sec. 3 treats the un-ordered
// traversal and other query shapes as easy variants of the ordered point
// query): children in fixed order, left then right, each entered
// only when the query region can reach its half-space.  The left subtree of a
// node holds coordinates <= its split value s in the split dimension, the
// right subtree coordinates >= s, so
//   radius (R2 = fl(r^2)): left is skipped iff sd = q[dim] - s > 0 and
//     fl(sd^2) > R2 (every left point then has d2 >= fl(sd^2) > R2), and
//     symmetrically for the right;
//   box [lo, hi]: left is skipped iff lo[dim] > s, right iff hi[dim] < s.
// Every point in the region is therefore processed, exactly once.  A lane
// counts them and keeps the `cap` best in a sorted list: by (d2, index) for
// radius queries (the kd_knn result within the radius), by caller index for
// box queries.  One "return to parent" level is fused as in the kNN step: a
// lane leaving a left child decides its parent's right child from the split
// stored in the child's record.
//
// With subtree bounding boxes (on request), a subtree is also tested when it
// is entered from its parent: it is left at once when its box and the query
// region are disjoint, and, for count-only queries (cap = 0), counted whole
// and left when its box lies inside the region.  Both tests are exact in
// binary32: rounding is monotone, so for every point p of a box and every
// dimension |fl(q - p)| lies between the offsets to the box's nearer and
// farther faces, and the left-to-right sum of squares of non-negative terms
// is monotone in each term; a point's d2 is therefore at least the box's
// smallest and at most its largest such sum.
namespace {

// Points in the subtree of node id `id` (a complete tree of N nodes in level
// order): the full width of every level below it, cut at N.
__device__ __forceinline__ uint32_t subtree_size(int32_t id, int32_t N) {
    uint32_t n = 0;
    int64_t lo = id, hi = id;
    while (lo <= N) {
        n += uint32_t((hi < N ? hi : N) - lo + 1);
        lo <<= 1;
        hi = (hi << 1) | 1;
    }
    return n;
}

struct RangeArgs {
    const void* nodes;      // TreeRec<D>[N + 2]
    const uint8_t* dims;    // stored split dimensions by node id (XD kernels), else NULL
    const float* sboxes;    // subtree bounding boxes [N + 2][box_words(D)] (SB kernels)
    int32_t box_below;      // boxes are tested for node ids below this
    int32_t N;
    const void* recs;       // NodeRec<D>[Q] Morton-sorted: the query point (radius) or the box centre
    const float* boxes;     // box queries: caller float [Q][2][D]
    uint32_t Q;
    float R2;               // radius queries
    int cap;                // results kept per query (0..K)
    int32_t* out_idx;       // [Q][cap] caller order
    float* out_d2;          // radius: [Q][cap] or NULL
    uint32_t* out_count;    // [Q]
    uint32_t* visited;      // [Q] entered nodes, or NULL
    uint32_t* counter;      // chunk cursor, zero at launch
    const int64_t* fill_off;  // fill mode: first output slot of each caller row
    int32_t* fill_idx;        // fill mode: every point in range, at fill_off[row] + its rank (NULL: off)
};

// The two query kinds as compile-time policies of one kernel: the paper's
// processNode and its "is this subtree in range" test passed as template
// parameters (Sec. 4 makes processNode a template parameter of the kernel).
// A policy holds a query's region and provides
//   load         the region of query slot r (its record; boxes by row),
//   shfl         the same region taken from another lane,
//   wants        which children of a node with split value sv (in the
//                dimension sel) the region reaches,
//   process      whether point c counts, and the high word of its list key,
//   empty_key    the key of an empty list slot,
//   box_test     a subtree's bounding box disjoint from / inside the region.
template <int D>
struct BallQuery {
    static constexpr bool kBox = false;
    float q[D];
    __device__ __forceinline__ void load(const NodeRec<D>& r, const float*) {
#pragma unroll
        for (int j = 0; j < D; ++j) q[j] = r.c[j];
    }
    __device__ __forceinline__ BallQuery shfl(int src) const {
        BallQuery o;
#pragma unroll
        for (int j = 0; j < D; ++j) o.q[j] = __shfl(q[j], src);
        return o;
    }
    // the left subtree holds coordinates <= sv, the right >= sv: a side is
    // skipped when the plane lies farther than the radius on the other side
    __device__ __forceinline__ void wants(const DimSel<D>& sel, float sv, float R2, bool& want_l,
                                          bool& want_r) const {
        const float sd = sel.template rot<0>(q) - sv;
        const bool far = sd * sd > R2;
        want_l = !(sd > 0.0f && far);
        want_r = !(sd < 0.0f && far);
    }
    // squared distance left to right without contraction, as kNN; the list
    // key is (d2, index)
    __device__ __forceinline__ bool process(const float (&c)[D], float R2, uint32_t& key_hi) const {
        float dx[D];
#pragma unroll
        for (int j = 0; j < D; ++j) dx[j] = q[j] - c[j];
        float d2 = dx[0] * dx[0];
#pragma unroll
        for (int j = 1; j < D; ++j) d2 = d2 + dx[j] * dx[j];
        key_hi = __float_as_uint(d2);
        return d2 <= R2;
    }
    static __device__ __forceinline__ uint64_t empty_key(float R2) { return make_key(R2, SENT_IDX); }
    // box lows w[0..D), highs w[H..H+D): the offsets to the nearer and the
    // farther face bound every point's |fl(q - p)| from below and above
    template <int H>
    __device__ __forceinline__ void box_test(const float (&w)[8], float R2, bool want_inside, bool& disjoint,
                                             bool& inside) const {
        float near[D], far[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float below = q[j] - w[j];      // >= 0 when q is above the low face
            const float above = q[j] - w[H + j];  // <= 0 when q is below the high face
            near[j] = below < 0.0f ? below : (above > 0.0f ? above : 0.0f);
            far[j] = fmaxf(fabsf(below), fabsf(above));
        }
        float dmin = near[0] * near[0], dmax = far[0] * far[0];
#pragma unroll
        for (int j = 1; j < D; ++j) {
            dmin = dmin + near[j] * near[j];
            dmax = dmax + far[j] * far[j];
        }
        disjoint = dmin > R2;
        inside = want_inside & (dmax <= R2);
    }
};

template <int D>
struct BoxQuery {
    static constexpr bool kBox = true;
    float lo[D], hi[D];
    __device__ __forceinline__ void load(const NodeRec<D>& r, const float* boxes) {
        const float* bx = boxes + size_t(r.idx) * 2 * D;  // the caller's box of this row
#pragma unroll
        for (int j = 0; j < D; ++j) {
            lo[j] = bx[j];
            hi[j] = bx[D + j];
        }
    }
    __device__ __forceinline__ BoxQuery shfl(int src) const {
        BoxQuery o;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            o.lo[j] = __shfl(lo[j], src);
            o.hi[j] = __shfl(hi[j], src);
        }
        return o;
    }
    __device__ __forceinline__ void wants(const DimSel<D>& sel, float sv, float, bool& want_l, bool& want_r) const {
        want_l = sel.template rot<0>(lo) <= sv;
        want_r = sel.template rot<0>(hi) >= sv;
    }
    // inside in every dimension, inclusive; the list key is (1, index), above
    // the spare slots' key 0
    __device__ __forceinline__ bool process(const float (&c)[D], float, uint32_t& key_hi) const {
        bool in = true;
#pragma unroll
        for (int j = 0; j < D; ++j) in = in & (lo[j] <= c[j]) & (c[j] <= hi[j]);
        key_hi = 1u;
        return in;
    }
    static __device__ __forceinline__ uint64_t empty_key(float) { return (uint64_t(2) << 32) | SENT_IDX; }
    template <int H>
    __device__ __forceinline__ void box_test(const float (&w)[8], float, bool want_inside, bool& disjoint,
                                             bool& inside) const {
        bool out = false, in = true;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            out = out | (w[H + j] < lo[j]) | (w[j] > hi[j]);
            in = in & (lo[j] <= w[j]) & (w[H + j] <= hi[j]);
        }
        disjoint = out;
        inside = want_inside & in;
    }
};

template <int D, int K, class Qy>
struct RangeLane {
    Qy g;              // the query region
    uint64_t L[K];
    int32_t curr, prev, row;
    uint32_t count, vis;
    int64_t base, end; // fill mode: the row's output slots [base, end)
};

template <int D, int K, class Qy>
__device__ __forceinline__ void range_finish(const RangeLane<D, K, Qy>& s, const RangeArgs& a) {
    a.out_count[s.row] = s.count;
    if (a.visited) a.visited[s.row] = s.vis;
    if (a.cap == 0) return;
    int32_t* oi = a.out_idx + int64_t(s.row) * a.cap;
    float* od = (!Qy::kBox && a.out_d2) ? a.out_d2 + int64_t(s.row) * a.cap : nullptr;
    const int off = K - a.cap;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= off) {
            const uint32_t id = uint32_t(s.L[j]);
            const bool empty = id == SENT_IDX;
            oi[j - off] = empty ? -1 : int32_t(id);
            if (od) od[j - off] = empty ? __builtin_inff() : key_d2(s.L[j]);
        }
    }
}

// The subtree of node `id` against the query region: disjoint (no point can
// be in range), or (count-only queries) wholly inside it.
template <int D, class Qy>
__device__ __forceinline__ void range_box_test(const Qy& g, const float* __restrict__ boxes, int32_t id, float R2,
                                               bool want_inside, bool& disjoint, bool& inside) {
    const uint4* p = reinterpret_cast<const uint4*>(boxes + int64_t(id) * box_words(D));
    float w[8];
    const uint4 u = p[0];
    w[0] = __uint_as_float(u.x); w[1] = __uint_as_float(u.y); w[2] = __uint_as_float(u.z); w[3] = __uint_as_float(u.w);
    w[4] = w[5] = w[6] = w[7] = 0.0f;
    if (box_words(D) == 8) {
        const uint4 v = p[1];
        w[4] = __uint_as_float(v.x); w[5] = __uint_as_float(v.y); w[6] = __uint_as_float(v.z); w[7] = __uint_as_float(v.w);
    }
    g.template box_test<box_words(D) / 2>(w, R2, want_inside, disjoint, inside);
}

template <int D, int K, class Qy, bool XD, bool SB>
__global__ __launch_bounds__(256) void range_persistent(RangeArgs a) {
    const TreeRec<D>* __restrict__ g1 = reinterpret_cast<const TreeRec<D>*>(a.nodes);
    const int32_t* __restrict__ ids = node_ids<D>(g1, a.N);
    const uint32_t lane = __lane_id();
    const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
    // chunk of 64 query slots held across the wave (lane l: slot cb + l)
    Qy chunk;
    int32_t crow = 0;
    uint32_t cb = 0, cn = 0, cpos = 0;
    bool exhausted = false;
    RangeLane<D, K, Qy> s;
    s.curr = 0;
    for (;;) {
        const uint64_t need = wave_ballot(s.curr == 0);
        if (need && !exhausted) {
            if (cpos == cn) {
                uint32_t c = 0;
                if (lane == 0) c = atomicAdd(a.counter, 64u);
                c = __builtin_amdgcn_readfirstlane(c);
                if (c >= a.Q) {
                    exhausted = true;
                } else {
                    cb = c;
                    cn = a.Q - c < 64u ? a.Q - c : 64u;
                    cpos = 0;
                    if (lane < cn) {
                        const NodeRec<D> r = load_query<D>(static_cast<const NodeRec<D>*>(a.recs) + cb + lane);
                        crow = r.idx;
                        chunk.load(r, a.boxes);
                    }
                }
            }
            if (!exhausted) {
                const uint32_t n = __popcll(need);
                const uint32_t rank = __popcll(need & lt_mask);
                const uint32_t take = n < cn - cpos ? n : cn - cpos;
                const int src = int(cpos + (rank < take ? rank : 0));
                const Qy vg = chunk.shfl(src);
                const int32_t vrow = __shfl(crow, src);
                if (s.curr == 0 && rank < take) {
                    s.g = vg;
                    s.row = vrow;
                    s.count = 0;
                    s.vis = 0;
                    s.base = a.fill_idx ? a.fill_off[vrow] : 0;
                    s.end = a.fill_idx ? a.fill_off[vrow + 1] : 0;
                    // spare slots (beyond cap) hold key 0 in front; empty
                    // slots the largest key of the list's kind
                    const uint64_t empty = Qy::empty_key(a.R2);
#pragma unroll
                    for (int j = 0; j < K; ++j) s.L[j] = (j < K - a.cap) ? uint64_t(0) : empty;
                    s.curr = 1;
                    s.prev = 0;
                }
                cpos += take;
            }
        }
        if (!wave_any(s.curr != 0)) break;
        if (s.curr != 0) {
            const int32_t curr = s.curr;
            float c[D];
            int32_t idx;
            float anc[rec_ancestors(D) > 0 ? rec_ancestors(D) : 1];
            load_tree<D>(g1 + curr, c, idx, anc);
            const uint32_t db = XD ? uint32_t(a.dims[curr]) : 0u;
            const bool from_parent = s.prev < curr;
            bool skip = false;
            if constexpr (SB) {
                if (from_parent && curr < a.box_below) {
                    bool disjoint, inside;
                    range_box_test<D>(s.g, a.sboxes, curr, a.R2, a.cap == 0, disjoint, inside);
                    if (inside) s.count += subtree_size(curr, a.N);
                    skip = disjoint | inside;
                }
            }
            if (from_parent & skip) ++s.vis;  // entered, and left at once
            if (from_parent & !skip) {
                ++s.vis;
                uint32_t key_hi;
                if (s.g.process(c, a.R2, key_hi)) {
                    const int32_t id = rec_has_idx(D) ? idx : ids[curr];
                    if (a.fill_idx && s.base + s.count < s.end) a.fill_idx[s.base + s.count] = id;
                    ++s.count;
                    const uint64_t key = (uint64_t(key_hi) << 32) | uint32_t(id);
                    if (key < s.L[K - 1]) list_insert<K>(s.L, key);
                }
            }
            const DimSel<D> sel = split_dim<D, XD, 0>(curr, db);
            bool want_l, want_r;
            s.g.wants(sel, sel.template rot<0>(c), a.R2, want_l, want_r);
            const int32_t lc = curr << 1, rc = lc | 1;
            int32_t next, nprev = curr;
            if (from_parent && !skip && want_l && lc <= a.N) next = lc;
            else if (((from_parent && !skip) || s.prev == lc) && want_r && rc <= a.N) next = rc;
            else {
                // return to the parent p; from a left child, p's right child
                // is decided here from p's split (stored in this record)
                const int32_t p = curr >> 1;
                next = p;
                if (p != 0 && (curr & 1) == 0) {
                    bool pl, pr;
                    s.g.wants(split_dim<D, XD, 1>(curr, db), anc[0], a.R2, pl, pr);
                    if (pr && (curr | 1) <= a.N) {
                        next = curr | 1;
                        nprev = p;
                    } else {
                        nprev = curr;  // p is done: the next trip returns from p
                        next = p;
                    }
                }
                if (next == p) {
                    // leave p: step to p's parent as coming back from p
                    nprev = p;
                    next = p >> 1;
                    if (p == 0) next = 0;
                }
            }
            s.prev = nprev;
            s.curr = next;
            if (next == 0) range_finish<D, K, Qy>(s, a);
        }
    }
}

// Centre of each box, (lo + hi) / 2 per dimension (the sort key only).
__global__ void box_centres(const float* __restrict__ boxes, int64_t Q, int D, float* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= Q * D) return;
    const int64_t q = i / D, j = i - q * D;
    out[i] = boxes[q * 2 * D + j] * 0.5f + boxes[q * 2 * D + D + j] * 0.5f;
}

template <int D, int K, bool XD>
void launch_range_kx(const RangeArgs& a, bool box, int grid, hipStream_t st) {
    const dim3 g(grid), b(256);
    if (a.sboxes) {
        if (box) hipLaunchKernelGGL((range_persistent<D, K, BoxQuery<D>, XD, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((range_persistent<D, K, BallQuery<D>, XD, true>), g, b, 0, st, a);
    } else {
        if (box) hipLaunchKernelGGL((range_persistent<D, K, BoxQuery<D>, XD, false>), g, b, 0, st, a);
        else hipLaunchKernelGGL((range_persistent<D, K, BallQuery<D>, XD, false>), g, b, 0, st, a);
    }
}

template <int D, int K>
hipError_t launch_range_k(const RangeArgs& a, bool box, int grid, hipStream_t st) {
    if (a.dims) launch_range_kx<D, K, true>(a, box, grid, st);
    else launch_range_kx<D, K, false>(a, box, grid, st);
    return hipGetLastError();
}

template <int D>
hipError_t launch_range(int K, const RangeArgs& a, bool box, int grid, hipStream_t st) {
    switch (K) {
        case 1: return launch_range_k<D, 1>(a, box, grid, st);
        case 2: return launch_range_k<D, 2>(a, box, grid, st);
        case 4: return launch_range_k<D, 4>(a, box, grid, st);
        case 8: return launch_range_k<D, 8>(a, box, grid, st);
        case 16: return launch_range_k<D, 16>(a, box, grid, st);
        case 32: return launch_range_k<D, 32>(a, box, grid, st);
        case 64: return launch_range_k<D, 64>(a, box, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

kd_status run_range(kd_tree t, const float* queries_or_boxes, int64_t Q, bool box, float R2, int cap,
                    int32_t* out_idx, float* out_d2, uint32_t* out_count, uint32_t* visited, bool planes_only,
                    kd_stream stream, const int64_t* fill_off, int32_t* fill_idx) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const DeviceInfo& dev = device_info(t->device);
    const int sort_bits = 16;
    void* ws = nullptr;
    // scratch: [counter | ...] query records, sort buffers, box centres
    const size_t qb = query_scratch_bytes(Q, t->dim, true, false, false);
    const size_t centre_bytes = box ? (size_t(Q) * t->dim * 4 + 255) & ~size_t(255) : 0;
    kd_status s = scratch(stream, qb + centre_bytes, &ws);
    if (s != KD_OK) return s;
    char* base = static_cast<char*>(ws);
    uint32_t* counter = reinterpret_cast<uint32_t*>(base);
    const size_t cursor_bytes = size_t(MAX_GROUPS) * CURSOR_STRIDE * 4;
    const size_t head = cursor_bytes + 4096;
    const size_t sq_bytes = (size_t(Q) * rec_bytes(t->dim) + 255) & ~size_t(255);
    void* sq = base + head;
    RangeArgs a = {};
    const float* keys = queries_or_boxes;
    if (box) {
        // boxes are ordered by their centres
        float* centres = reinterpret_cast<float*>(base + qb);
        const int64_t n = Q * t->dim;
        hipLaunchKernelGGL(box_centres, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, queries_or_boxes, Q,
                           t->dim, centres);
        KD_HIP(hipGetLastError());
        keys = centres;
        a.boxes = queries_or_boxes;
    }
    // Morton order (the first sort kernel clears the counter)
    hipEvent_t evs;
    s = timing_begin(st, &evs);
    if (s != KD_OK) return s;
    s = reorder_queries(t, keys, Q, sort_bits, base + head + sq_bytes, sq, counter, 64, st);
    if (s != KD_OK) return s;
    s = timing_end(st, evs, "sort");
    if (s != KD_OK) return s;
    a.recs = sq;
    a.nodes = t->d_nodes;
    a.dims = t->d_dims;
    a.sboxes = planes_only ? nullptr : static_cast<const float*>(t->d_boxes);
    a.box_below = box_id_limit(t->N);
    a.N = int32_t(t->N);
    a.Q = uint32_t(Q);
    a.R2 = R2;
    a.cap = cap;
    a.out_idx = out_idx;
    a.out_d2 = out_d2;
    a.out_count = out_count;
    a.visited = visited;
    a.counter = counter;
    a.fill_off = fill_off;
    a.fill_idx = fill_idx;
    const int K = cap > 0 ? k_template(cap) : 1;
    int64_t grid = int64_t(dev.cus) * 6;  // 24 waves per CU
    const int64_t need = (Q + 255) / 256;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipEvent_t ev0;
    s = timing_begin(st, &ev0);
    if (s != KD_OK) return s;
    hipError_t e = t->dim == 2 ? launch_range<2>(K, a, box, int(grid), st)
                 : t->dim == 3 ? launch_range<3>(K, a, box, int(grid), st) : launch_range<4>(K, a, box, int(grid), st);
    if (e != hipSuccess) return hip_error(e, "range query launch");
    return timing_end(st, ev0, box ? "box" : "radius");
}

}  // namespace kd
