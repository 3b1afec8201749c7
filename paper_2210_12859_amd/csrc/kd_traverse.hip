// kd_traverse.hip -- stack-free fcp / kNN traversal kernels for gfx950.
//
// Each lane runs the two-integer state machine of the paper's Sec. 3.2 for
// one query: `curr` and `prev` alone decide where to go next.
//   * first visit (prev < curr, i.e. we came from the parent): process the
//     node -- squared distance, insertion into the k-best list, which may
//     shrink the search radius -- then step to the close child;
//   * second visit (prev == close child): step to the far child if its
//     subtree is still in range, else to the parent;
//   * third visit (prev == far child): step to the parent;
//   * the root stepping to its parent (-1) ends the traversal.
// The close child is the right child iff q[dim] - split > 0 (Sec. 3.2).  The
// far-range test is taken in squared form, fl(sd*sd) <= worst d2 of the list,
// non-strict: every point of the far subtree has d2 >= fl(sd*sd), so the test
// never prunes a point that could enter the list, ties included.
//
// Visits to children that do not exist (index >= N) are resolved in the same
// loop trip instead of stepping there and bouncing back: the next node is
// chosen exactly as the bounce would have chosen it, so the processed-node
// sequence equals the paper's (and the ordered recursion's).
//
// MI355X mapping
//   * persistent grid; each wave pulls chunks of 64 sorted query slots from
//     a global counter; lanes whose query finished are refilled under one
//     wave-uniform branch (ballot + mbcnt), so waves stay full;
//   * the top tree levels are staged in LDS once per workgroup;
//   * nodes are 16-byte records (x, y, z, caller index) for D=3: one dwordx4
//     load per loop trip gives the split coordinate, the point and its index;
//   * the k-best list lives in VGPRs as 64-bit keys (d2 bits << 32 | index),
//     so the lexicographic (d2, index) order is one unsigned compare (d2 >= 0,
//     and the bit pattern of a non-negative float is monotone); insertion is
//     a fixed, fully unrolled network behind a wave-uniform skip.
#include <hip/hip_runtime.h>

#include "kd_internal.h"

namespace kd {

namespace {

constexpr uint32_t SENT_IDX = 0x7fffffffu;

struct TravArgs {
    const void* nodes;       // NodeRec<D>[N]
    int32_t N;
    int32_t lds_nodes;       // records staged in LDS (a prefix of the array)
    const float* queries;    // caller [Q][D]
    const int32_t* perm;     // slot -> caller row; NULL = identity
    uint32_t Q;              // query slots
    int k;                   // requested k (<= K)
    float R2;                // fl32(maxRadius^2)
    int32_t* out_idx;        // [Q][k] caller order
    float* out_d2;           // [Q][k] or NULL
    uint32_t* visited;       // [Q] or NULL
    uint32_t* counter;       // work-queue cursor, zero at launch
};

__device__ __forceinline__ uint64_t make_key(float d2, int32_t idx) {
    return (uint64_t(__float_as_uint(d2)) << 32) | uint32_t(idx);
}

__device__ __forceinline__ float key_d2(uint64_t key) { return __uint_as_float(uint32_t(key >> 32)); }

// Sorted insertion of `key` (known to be < L[K-1]) into the ascending list L.
template <int K>
__device__ __forceinline__ void list_insert(uint64_t (&L)[K], uint64_t key) {
#pragma unroll
    for (int j = K - 1; j > 0; --j) {
        const bool lt_prev = key < L[j - 1];
        const bool lt_here = key < L[j];
        L[j] = lt_prev ? L[j - 1] : (lt_here ? key : L[j]);
    }
    L[0] = key < L[0] ? key : L[0];
}

template <int D>
__device__ __forceinline__ NodeRec<D> load_node(const NodeRec<D>* __restrict__ g, const NodeRec<D>* l,
                                                int32_t curr, int32_t lds_nodes) {
    NodeRec<D> r;
    if (curr < lds_nodes) {
        r = l[curr];
    } else {
        r = g[curr];
    }
    return r;
}

template <int D>
__device__ __forceinline__ int dim_step(int dim, bool down) {
    int d = dim + (down ? 1 : D - 1);
    return d >= D ? d - D : d;
}

// Per-lane query state.
template <int D, int K>
struct Lane {
    float q[D];
    uint64_t L[K];
    int32_t curr, prev;
    int dim;
    uint32_t slot;
    uint32_t vis;
};

template <int D, int K>
__device__ __forceinline__ void lane_start(Lane<D, K>& s, const TravArgs& a, uint32_t slot) {
    s.slot = slot;
    const int32_t row = a.perm ? a.perm[slot] : int32_t(slot);
#pragma unroll
    for (int j = 0; j < D; ++j) s.q[j] = a.queries[int64_t(row) * D + j];
    // Slots beyond k hold the smallest key so the list's worst entry is the
    // k-th real one; real keys are >= 0 and never move in front of them.
    const uint64_t sent = make_key(a.R2, SENT_IDX);
#pragma unroll
    for (int j = 0; j < K; ++j) s.L[j] = (j < K - a.k) ? uint64_t(0) : sent;
    s.curr = 0;
    s.prev = -1;
    s.dim = 0;
    s.vis = 0;
}

template <int D, int K, bool COUNT>
__device__ __forceinline__ void lane_finish(const Lane<D, K>& s, const TravArgs& a) {
    const int32_t row = a.perm ? a.perm[s.slot] : int32_t(s.slot);
    int32_t* oi = a.out_idx + int64_t(row) * a.k;
    float* od = a.out_d2 ? a.out_d2 + int64_t(row) * a.k : nullptr;
    const int off = K - a.k;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= off) {
            const uint32_t id = uint32_t(s.L[j]);
            const bool empty = id == SENT_IDX;
            oi[j - off] = empty ? -1 : int32_t(id);
            if (od) od[j - off] = empty ? __builtin_inff() : key_d2(s.L[j]);
        }
    }
    if (COUNT && a.visited) a.visited[row] = s.vis;
}

// One trip of the state machine.  Returns the next node (-1 = finished).
template <int D, int K, bool COUNT>
__device__ __forceinline__ int32_t lane_step(Lane<D, K>& s, const NodeRec<D>* __restrict__ g,
                                             const NodeRec<D>* l, int32_t N, int32_t lds_nodes) {
    const int32_t curr = s.curr;
    const NodeRec<D> r = load_node<D>(g, l, curr, lds_nodes);
    float dx[D];
#pragma unroll
    for (int j = 0; j < D; ++j) dx[j] = s.q[j] - r.c[j];
    float sd = dx[0];
#pragma unroll
    for (int j = 1; j < D; ++j) sd = (s.dim == j) ? dx[j] : sd;

    const bool from_parent = s.prev < curr;
    if (from_parent) {
        // processNode: exact binary32 squared distance, left to right.
        float d2 = dx[0] * dx[0];
#pragma unroll
        for (int j = 1; j < D; ++j) d2 = d2 + dx[j] * dx[j];
        const uint64_t key = make_key(d2, r.idx);
        if (COUNT) s.vis++;
        if (key < s.L[K - 1]) list_insert<K>(s.L, key);
    }
    const float worst = key_d2(s.L[K - 1]);
    const bool far_in = sd * sd <= worst;
    const int32_t close_side = sd > 0.0f ? 1 : 0;
    const int32_t close_c = 2 * curr + 1 + close_side;
    const int32_t far_c = 2 * curr + 2 - close_side;
    const int32_t parent = (curr - 1) >> 1;  // -1 for the root
    const bool close_ok = close_c < N;
    const bool try_far = from_parent ? !close_ok : (s.prev == close_c);
    const bool go_close = from_parent && close_ok;
    const bool go_far = try_far && far_in && far_c < N;
    const int32_t next = go_close ? close_c : (go_far ? far_c : parent);
    s.dim = dim_step<D>(s.dim, go_close || go_far);
    s.prev = curr;
    s.curr = next;
    return next;
}

template <int D, int K, bool COUNT>
__global__ __launch_bounds__(256) void knn_persistent(TravArgs a) {
    extern __shared__ unsigned char smem_raw[];
    NodeRec<D>* lnodes = reinterpret_cast<NodeRec<D>*>(smem_raw);
    const NodeRec<D>* __restrict__ g = reinterpret_cast<const NodeRec<D>*>(a.nodes);
    for (int i = threadIdx.x; i < a.lds_nodes; i += blockDim.x) lnodes[i] = g[i];
    __syncthreads();

    const uint32_t lane = __lane_id();
    // wave-private reservoir of query slots [rbase, rbase + rleft)
    uint32_t rbase = 0, rleft = 0;
    if (lane == 0) rbase = atomicAdd(a.counter, 64u);
    rbase = __builtin_amdgcn_readfirstlane(rbase);
    rleft = 64;

    Lane<D, K> s;
    bool active = rbase + lane < a.Q;
    if (active) lane_start<D, K>(s, a, rbase + lane);
    rbase += 64;
    rleft = 0;

    while (__builtin_amdgcn_read_exec() != 0 && __any(active)) {
        bool done = false;
        if (active) {
            const int32_t next = lane_step<D, K, COUNT>(s, g, lnodes, a.N, a.lds_nodes);
            done = next < 0;
        }
        const uint64_t dmask = __ballot(done);
        if (dmask) {
            if (done) lane_finish<D, K, COUNT>(s, a);
            const uint32_t n = __popcll(dmask);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(uint32_t(dmask >> 32),
                                                           __builtin_amdgcn_mbcnt_lo(uint32_t(dmask), 0u));
            uint32_t nb = 0;
            if (rleft < n) {
                if (lane == 0) nb = atomicAdd(a.counter, 64u);
                nb = __builtin_amdgcn_readfirstlane(nb);
            }
            if (done) {
                const uint32_t slot = rank < rleft ? rbase + rank : nb + (rank - rleft);
                active = slot < a.Q;
                if (active) lane_start<D, K>(s, a, slot);
            }
            if (rleft < n) {
                rbase = nb + (n - rleft);
                rleft = 64 - (n - rleft);
            } else {
                rbase += n;
                rleft -= n;
            }
        }
    }
}

__global__ void zero_u32(uint32_t* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <int D, int K, bool COUNT>
hipError_t launch_knn(const TravArgs& a, int block, int grid, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL((knn_persistent<D, K, COUNT>), dim3(grid), dim3(block), lds_bytes, st, a);
    return hipGetLastError();
}

template <int D, bool COUNT>
hipError_t dispatch_k(int K, const TravArgs& a, int block, int grid, size_t lds, hipStream_t st) {
    switch (K) {
        case 1: return launch_knn<D, 1, COUNT>(a, block, grid, lds, st);
        case 2: return launch_knn<D, 2, COUNT>(a, block, grid, lds, st);
        case 4: return launch_knn<D, 4, COUNT>(a, block, grid, lds, st);
        case 8: return launch_knn<D, 8, COUNT>(a, block, grid, lds, st);
        case 16: return launch_knn<D, 16, COUNT>(a, block, grid, lds, st);
        case 32: return launch_knn<D, 32, COUNT>(a, block, grid, lds, st);
        case 64: return launch_knn<D, 64, COUNT>(a, block, grid, lds, st);
    }
    return hipErrorInvalidValue;
}

template <bool COUNT>
hipError_t dispatch_dk(int D, int K, const TravArgs& a, int block, int grid, size_t lds, hipStream_t st) {
    switch (D) {
        case 2: return dispatch_k<2, COUNT>(K, a, block, grid, lds, st);
        case 3: return dispatch_k<3, COUNT>(K, a, block, grid, lds, st);
        case 4: return dispatch_k<4, COUNT>(K, a, block, grid, lds, st);
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

}  // namespace

int k_template(int k) {
    int K = 1;
    while (K < k) K <<= 1;
    return K;
}

kd_status run_knn(kd_tree t, const float* queries, int64_t Q, const QueryPlan& plan,
                  int32_t* out_idx, float* out_d2, uint32_t* visited, kd_stream stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const DeviceInfo& dev = device_info(t->device);
    void* ws = nullptr;
    kd_status s = scratch(stream, 256, &ws);
    if (s != KD_OK) return s;
    uint32_t* counter = reinterpret_cast<uint32_t*>(ws);
    hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, counter, 1);
    KD_HIP(hipGetLastError());

    TravArgs a;
    a.nodes = t->d_nodes;
    a.N = int32_t(t->N);
    int64_t lds_nodes = (int64_t(1) << plan.lds_levels) - 1;
    if (lds_nodes > t->N) lds_nodes = t->N;
    size_t lds_bytes = size_t(lds_nodes) * rec_bytes(t->dim);
    if (lds_bytes > size_t(dev.lds_bytes)) return set_error(KD_EINVAL, "lds_levels too large for LDS");
    a.lds_nodes = int32_t(lds_nodes);
    a.queries = queries;
    a.perm = nullptr;
    a.Q = uint32_t(Q);
    a.k = plan.k;
    a.R2 = plan.R2;
    a.out_idx = out_idx;
    a.out_d2 = out_d2;
    a.visited = visited;
    a.counter = counter;

    const int block = plan.block;
    const int waves_per_block = block / 64;
    int64_t grid = int64_t(dev.cus) * plan.waves_per_cu / waves_per_block;
    const int64_t need = (Q + block - 1) / block;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipEvent_t ev0;
    s = timing_begin(st, &ev0);
    if (s != KD_OK) return s;
    hipError_t e = visited ? dispatch_dk<true>(t->dim, plan.K, a, block, int(grid), lds_bytes, st)
                           : dispatch_dk<false>(t->dim, plan.K, a, block, int(grid), lds_bytes, st);
    if (e != hipSuccess) return hip_error(e, "knn_persistent launch");
    return timing_end(st, ev0, "traverse");
}

}  // namespace kd
