// kd_build_gpu.hip -- the canonical left-balanced k-d tree built on the GPU.
//
// The tree is the one every correct builder produces (Sec. 4): at level-order
// position n (split dimension floor(log2(n+1)) mod D) sits the element of
// rank leftSize(|S|) of the node's subtree set S, ordered by (split
// coordinate, caller index); smaller elements form the left subtree, larger
// ones the right.
//
// Level by level.  Every point not yet placed belongs to one node of the
// current level (its segment).  For each dimension d the points are sorted
// once by (coordinate d, caller index) into the list L_d (a stable radix sort
// of the coordinates, starting from caller order).  At level l with split
// dimension d, a stable radix sort of L_d by segment (placed points last)
// lists every segment's points in (coordinate, index) order, contiguously and
// in level order.  The segments' sizes and starts follow from N alone (the
// tree is complete): with W = 2^(H-1-l) last-level slots under each node of
// level l and `last` nodes on the last level, segment s starts at
// s (W - 1) + min(last, s W) and holds (W - 1) + clamp(last - s W, 0, W)
// points.  The point at offset leftSize(size) of segment s is placed at
// position 2^l - 1 + s; the others move to segment 2s (left child) or 2s + 1
// (right child) of the next level.  H levels, each a sort of N keys on l + 1
// bits.  The result equals the host builder's and the oracle's byte for byte.
//
// Stored split dimensions (the widest rule): every segment of the level
// picks its own dimension, so all D lists are sorted by segment each level.
// In list L_d a segment's points are in coordinate order, so its extent in d
// is the coordinate of its last point minus that of its first; the largest
// extent (the lowest d on ties) is the segment's dimension, and its points
// are ranked in that dimension's list.  Each point is assigned once, by the
// list of its segment's dimension.  H levels of D sorts.
//
// Node records and subtree boxes are then written on the device as well.
#include <hip/hip_runtime.h>

#include "kd_internal.h"

namespace kd {

namespace {

constexpr uint32_t PLACED = 0xffffffffu;

// Radix key of a coordinate: unsigned order equals float order (-0 == +0).
__device__ __forceinline__ uint32_t coord_key(float f) {
    uint32_t b = __float_as_uint(f);
    if (b == 0x80000000u) b = 0;  // -0 orders as +0, ties then go by index
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Size of the left subtree of a complete tree of n nodes (the rank of the
// subtree root in its ordered set).
__device__ __forceinline__ int64_t left_size_dev(int64_t n) {
    if (n < 2) return 0;
    const int h = 63 - __builtin_clzll(uint64_t(n));   // n has h + 1 levels
    const int64_t full_above = (int64_t(1) << h) - 1;  // nodes above the last level
    const int64_t on_last = n - full_above;
    const int64_t half = int64_t(1) << (h - 1);        // last-level slots under the left child
    return (half - 1) + (on_last < half ? on_last : half);
}

__global__ void dim_keys(const float* __restrict__ pts, uint32_t N, int D, int d, uint32_t* __restrict__ k,
                         uint32_t* __restrict__ v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    k[i] = coord_key(pts[size_t(i) * D + d]);
    v[i] = i;
}

__global__ void fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void level_keys(const uint32_t* __restrict__ Ld, const uint32_t* __restrict__ seg, uint32_t N,
                           uint32_t placed_key, uint32_t* __restrict__ k, uint32_t* __restrict__ v) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const uint32_t p = Ld[j];
    const uint32_t s = seg[p];
    k[j] = s == PLACED ? placed_key : s;
    v[j] = p;
}

// Points of level `level`'s segments in (segment, coordinate, index) order:
// place each segment's root, send the rest to the child segments.
__global__ void level_assign(const uint32_t* __restrict__ k, const uint32_t* __restrict__ v, uint32_t R,
                             int64_t W, int64_t last, int64_t first, int32_t* __restrict__ order,
                             uint32_t* __restrict__ seg) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= R) return;
    const int64_t s = k[j];
    const uint32_t p = v[j];
    const int64_t sW = s * W;
    const int64_t start = s * (W - 1) + (last < sW ? last : sW);
    int64_t extra = last - sW;
    extra = extra < 0 ? 0 : (extra > W ? W : extra);
    const int64_t size = (W - 1) + extra;
    const int64_t m = left_size_dev(size);
    const int64_t o = int64_t(j) - start;
    if (o == m) {
        order[first + s] = int32_t(p);
        seg[p] = PLACED;
    } else {
        seg[p] = uint32_t(o < m ? 2 * s : 2 * s + 1);
    }
}

// Split dimension of each node of the level (widest rule): the extent of
// segment s in d is the coordinate of its last point minus its first's in
// the segment-sorted list S_d.
__global__ void segment_dims(const float* __restrict__ pts, int D, const uint32_t* __restrict__ S0,
                             const uint32_t* __restrict__ S1, const uint32_t* __restrict__ S2,
                             const uint32_t* __restrict__ S3, uint32_t nseg, int64_t W, int64_t last, int64_t first,
                             uint8_t* __restrict__ segdim, uint8_t* __restrict__ pos_dims) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int64_t sW = int64_t(s) * W;
    const int64_t start = int64_t(s) * (W - 1) + (last < sW ? last : sW);
    int64_t extra = last - sW;
    extra = extra < 0 ? 0 : (extra > W ? W : extra);
    const int64_t size = (W - 1) + extra;  // >= 1: node first + s exists
    const uint32_t* S[4] = {S0, S1, S2, S3};
    int best = 0;
    float best_ext = -1.0f;
    for (int d = 0; d < D; ++d) {
        const float lo = pts[size_t(S[d][start]) * D + d];
        const float hi = pts[size_t(S[d][start + size - 1]) * D + d];
        const float ext = hi - lo;
        if (ext > best_ext) {
            best_ext = ext;
            best = d;
        }
    }
    segdim[s] = uint8_t(best);
    pos_dims[first + s] = uint8_t(best);
}

// level_assign for the points of list d whose segment splits in d; the new
// segments go to seg_next (seg is still read by the other lists' launches).
__global__ void level_assign_widest(const uint32_t* __restrict__ S, int d, const uint8_t* __restrict__ segdim,
                                    const uint32_t* __restrict__ seg, uint32_t R, int64_t W, int64_t last,
                                    int64_t first, int32_t* __restrict__ order, uint32_t* __restrict__ seg_next) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= R) return;
    const uint32_t p = S[j];
    const int64_t s = seg[p];  // unplaced: the first R entries of the list
    if (segdim[s] != d) return;
    const int64_t sW = s * W;
    const int64_t start = s * (W - 1) + (last < sW ? last : sW);
    int64_t extra = last - sW;
    extra = extra < 0 ? 0 : (extra > W ? W : extra);
    const int64_t size = (W - 1) + extra;
    const int64_t m = left_size_dev(size);
    const int64_t o = int64_t(j) - start;
    if (o == m) {
        order[first + s] = int32_t(p);
        seg_next[p] = PLACED;
    } else {
        seg_next[p] = uint32_t(o < m ? 2 * s : 2 * s + 1);
    }
}

// Per node id: the split dimensions of the node and its three nearest
// ancestors, 2 bits each (own dimension in bits 0-1).
__global__ void pack_dims(const uint8_t* __restrict__ pos_dims, uint32_t N, uint8_t* __restrict__ out) {
    const uint32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= N) return;
    uint32_t a = pos + 1, b = 0;
    for (int m = 0; m < 4 && a >= 1; ++m, a >>= 1) b |= uint32_t(pos_dims[a - 1]) << (2 * m);
    out[pos + 1] = uint8_t(b);
}

// Any non-finite coordinate sets *bad.
__global__ void check_finite(const float* __restrict__ pts, size_t n, uint32_t* __restrict__ bad) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        if (!__builtin_isfinite(pts[i])) *bad = 1u;
}

// Node record of id pos + 1 (see TreeRec): coordinates, caller index (in the
// record or in the index array), ancestor splits (parent first).
template <int D>
__global__ void pack_records_dev(const float* __restrict__ pts, const int32_t* __restrict__ order, uint32_t N,
                                 const uint8_t* __restrict__ pos_dims, TreeRec<D>* __restrict__ r) {
    const uint32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= N) return;
    constexpr int A0 = D + (rec_has_idx(D) ? 1 : 0);
    TreeRec<D> rec;
#pragma unroll
    for (int w = 0; w < rec_words(D); ++w) rec.w[w] = 0;
    const int32_t i = order[pos];
#pragma unroll
    for (int j = 0; j < D; ++j) rec.w[j] = __float_as_uint(pts[size_t(i) * D + j]);
    if constexpr (rec_has_idx(D)) rec.w[D] = uint32_t(i);
    else reinterpret_cast<int32_t*>(r + (size_t(N) + 2))[pos + 1] = i;
    uint32_t a = (pos + 1) >> 1;
#pragma unroll
    for (int m = 0; m < rec_ancestors(D); ++m) {
        if (a >= 1) {
            const int lvl = 31 - __builtin_clz(a);
            const int d = pos_dims ? int(pos_dims[a - 1]) : lvl % D;
            rec.w[A0 + m] = __float_as_uint(pts[size_t(order[a - 1]) * D + d]);
        }
        a >>= 1;
    }
    r[pos + 1] = rec;
}

// Bounding boxes of the subtrees of node ids [lo, hi] (one level): the own
// point and the children's boxes (computed by the previous launch).
__global__ void boxes_level(const float* __restrict__ pts, const int32_t* __restrict__ order, uint32_t N, int D,
                            uint32_t lo, uint32_t hi, float* __restrict__ boxes) {
    const uint32_t id = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (id > hi) return;
    const int BW = D == 2 ? 4 : 8, H = BW / 2;
    float* b = boxes + size_t(id) * BW;
    const float* p = pts + size_t(order[id - 1]) * D;
    float mn[4], mx[4];
    for (int j = 0; j < D; ++j) mn[j] = mx[j] = p[j];
    for (uint32_t c = 2 * id; c <= 2 * id + 1 && c <= N; ++c) {
        const float* cb = boxes + size_t(c) * BW;
        for (int j = 0; j < D; ++j) {
            // keep the current value unless the child's is strictly beyond it
            // (the host builder's rule, so -0 / +0 come out the same)
            mn[j] = cb[j] < mn[j] ? cb[j] : mn[j];
            mx[j] = mx[j] < cb[H + j] ? cb[H + j] : mx[j];
        }
    }
    for (int j = 0; j < D; ++j) {
        b[j] = mn[j];
        b[H + j] = mx[j];
    }
}

inline dim3 grid_for(uint64_t n) { return dim3(unsigned((n + 255) / 256)); }

}  // namespace

namespace {
kd_status build_widest_device(const float* d_pts, int64_t N, int D, int32_t* d_order, uint8_t* d_pos_dims,
                              hipStream_t st) {
    const uint32_t n = uint32_t(N);
    const size_t b4 = (size_t(n) * 4 + 255) & ~size_t(255);
    const size_t b1 = (size_t(n) + 255) & ~size_t(255);
    const size_t hist_b = (sort_pairs_scratch_bytes(n) + 255) & ~size_t(255);
    // seg | seg_next | L_0 .. L_{D-1} | S_0 .. S_{D-1} | k0 v0 k1 v1 | segdim | histograms
    char* ws = nullptr;
    KD_HIP(hipMalloc(&ws, b4 * (2 + 2 * size_t(D) + 4) + b1 + hist_b));
    struct Free {
        char* p;
        ~Free() { (void)hipFree(p); }
    } guard{ws};
    uint32_t* seg = reinterpret_cast<uint32_t*>(ws);
    uint32_t* seg_next = reinterpret_cast<uint32_t*>(ws + b4);
    uint32_t* L[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t* S[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int d = 0; d < D; ++d) {
        L[d] = reinterpret_cast<uint32_t*>(ws + b4 * (2 + d));
        S[d] = reinterpret_cast<uint32_t*>(ws + b4 * (2 + D + d));
    }
    char* tail = ws + b4 * (2 + 2 * size_t(D));
    uint32_t* k0 = reinterpret_cast<uint32_t*>(tail);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(tail + b4);
    uint32_t* k1 = reinterpret_cast<uint32_t*>(tail + 2 * b4);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(tail + 3 * b4);
    uint8_t* segdim = reinterpret_cast<uint8_t*>(tail + 4 * b4);
    void* hist = tail + 4 * b4 + b1;
    const dim3 g = grid_for(n), b(256);
    for (int d = 0; d < D; ++d) {
        hipLaunchKernelGGL(dim_keys, g, b, 0, st, d_pts, n, D, d, k0, v0);
        KD_HIP(hipGetLastError());
        bool second = false;
        kd_status s = sort_pairs(k0, v0, k1, v1, n, 32, hist, st, &second);
        if (s != KD_OK) return s;
        KD_HIP(hipMemcpyAsync(L[d], second ? v1 : v0, size_t(n) * 4, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(fill_u32, g, b, 0, st, seg, n, 0u);
    KD_HIP(hipGetLastError());
    int H = 0;
    while (H < 31 && (int64_t(1) << H) <= N) ++H;
    const int64_t last = N - ((int64_t(1) << (H - 1)) - 1);
    for (int l = 0; l < H; ++l) {
        const int64_t first = (int64_t(1) << l) - 1;
        const uint32_t R = uint32_t(N - first);
        const int64_t W = int64_t(1) << (H - 1 - l);
        for (int d = 0; d < D; ++d) {
            hipLaunchKernelGGL(level_keys, g, b, 0, st, L[d], seg, n, uint32_t(1) << l, k0, v0);
            KD_HIP(hipGetLastError());
            bool second = false;
            kd_status s = sort_pairs(k0, v0, k1, v1, n, l + 1, hist, st, &second);
            if (s != KD_OK) return s;
            KD_HIP(hipMemcpyAsync(S[d], second ? v1 : v0, size_t(R) * 4, hipMemcpyDeviceToDevice, st));
        }
        const int64_t nodes = std::min<int64_t>(int64_t(1) << l, N - first);
        hipLaunchKernelGGL(segment_dims, grid_for(uint64_t(nodes)), b, 0, st, d_pts, D, S[0], S[1], S[2], S[3],
                           uint32_t(nodes), W, last, first, segdim, d_pos_dims);
        KD_HIP(hipGetLastError());
        KD_HIP(hipMemcpyAsync(seg_next, seg, size_t(n) * 4, hipMemcpyDeviceToDevice, st));
        for (int d = 0; d < D; ++d) {
            hipLaunchKernelGGL(level_assign_widest, grid_for(R), b, 0, st, S[d], d, segdim, seg, R, W, last, first,
                               d_order, seg_next);
            KD_HIP(hipGetLastError());
        }
        std::swap(seg, seg_next);
    }
    KD_HIP(hipStreamSynchronize(st));  // the workspace is freed on return
    return KD_OK;
}
}  // namespace

kd_status build_level_order_device(const float* d_pts, int64_t N, int D, int32_t* d_order, hipStream_t st,
                                   uint8_t* d_pos_dims) {
    if (N <= 0) return KD_OK;
    if (d_pos_dims) return build_widest_device(d_pts, N, D, d_order, d_pos_dims, st);
    const uint32_t n = uint32_t(N);
    const size_t b4 = (size_t(n) * 4 + 255) & ~size_t(255);
    const size_t hist_b = (sort_pairs_scratch_bytes(n) + 255) & ~size_t(255);
    // seg | L_0 .. L_{D-1} | k0 v0 k1 v1 | histograms
    char* ws = nullptr;
    KD_HIP(hipMalloc(&ws, b4 * (1 + size_t(D) + 4) + hist_b));
    struct Free {
        char* p;
        ~Free() { (void)hipFree(p); }
    } guard{ws};
    uint32_t* seg = reinterpret_cast<uint32_t*>(ws);
    uint32_t* L[4];
    for (int d = 0; d < D; ++d) L[d] = reinterpret_cast<uint32_t*>(ws + b4 * (1 + d));
    uint32_t* k0 = reinterpret_cast<uint32_t*>(ws + b4 * (1 + D));
    uint32_t* v0 = reinterpret_cast<uint32_t*>(ws + b4 * (2 + D));
    uint32_t* k1 = reinterpret_cast<uint32_t*>(ws + b4 * (3 + D));
    uint32_t* v1 = reinterpret_cast<uint32_t*>(ws + b4 * (4 + D));
    void* hist = ws + b4 * (5 + D);
    const dim3 g = grid_for(n), b(256);

    // L_d: caller indices in (coordinate d, index) order (stable sort from
    // caller order)
    for (int d = 0; d < D; ++d) {
        hipLaunchKernelGGL(dim_keys, g, b, 0, st, d_pts, n, D, d, k0, v0);
        KD_HIP(hipGetLastError());
        bool second = false;
        kd_status s = sort_pairs(k0, v0, k1, v1, n, 32, hist, st, &second);
        if (s != KD_OK) return s;
        KD_HIP(hipMemcpyAsync(L[d], second ? v1 : v0, size_t(n) * 4, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(fill_u32, g, b, 0, st, seg, n, 0u);
    KD_HIP(hipGetLastError());

    int H = 0;  // levels: floor(log2 N) + 1
    while (H < 31 && (int64_t(1) << H) <= N) ++H;
    const int64_t last = N - ((int64_t(1) << (H - 1)) - 1);  // nodes on the last level
    for (int l = 0; l < H; ++l) {
        const int d = l % D;
        const int64_t first = (int64_t(1) << l) - 1;
        const uint32_t R = uint32_t(N - first);  // points not yet placed
        hipLaunchKernelGGL(level_keys, g, b, 0, st, L[d], seg, n, uint32_t(1) << l, k0, v0);
        KD_HIP(hipGetLastError());
        bool second = false;
        kd_status s = sort_pairs(k0, v0, k1, v1, n, l + 1, hist, st, &second);
        if (s != KD_OK) return s;
        const int64_t W = int64_t(1) << (H - 1 - l);
        hipLaunchKernelGGL(level_assign, grid_for(R), b, 0, st, second ? k1 : k0, second ? v1 : v0, R, W, last,
                           first, d_order, seg);
        KD_HIP(hipGetLastError());
    }
    KD_HIP(hipStreamSynchronize(st));  // the workspace is freed on return
    return KD_OK;
}

kd_status pack_tree_device(const float* d_pts, const int32_t* d_order, int64_t N, int D, void* d_nodes,
                           float* d_boxes, hipStream_t st, const uint8_t* d_pos_dims, uint8_t* d_dims) {
    if (N <= 0) return KD_OK;
    const uint32_t n = uint32_t(N);
    KD_HIP(hipMemsetAsync(d_nodes, 0, node_buffer_bytes(D, N), st));
    KD_HIP(hipMemsetAsync(d_boxes, 0, box_buffer_bytes(D, N), st));
    const dim3 g = grid_for(n), b(256);
    switch (D) {
        case 2:
            hipLaunchKernelGGL(pack_records_dev<2>, g, b, 0, st, d_pts, d_order, n, d_pos_dims, (TreeRec<2>*)d_nodes);
            break;
        case 3:
            hipLaunchKernelGGL(pack_records_dev<3>, g, b, 0, st, d_pts, d_order, n, d_pos_dims, (TreeRec<3>*)d_nodes);
            break;
        default:
            hipLaunchKernelGGL(pack_records_dev<4>, g, b, 0, st, d_pts, d_order, n, d_pos_dims, (TreeRec<4>*)d_nodes);
            break;
    }
    KD_HIP(hipGetLastError());
    if (d_dims) {
        KD_HIP(hipMemsetAsync(d_dims, 0, size_t(N) + 2, st));
        hipLaunchKernelGGL(pack_dims, g, b, 0, st, d_pos_dims, n, d_dims);
        KD_HIP(hipGetLastError());
    }
    int H = 0;
    while (H < 31 && (int64_t(1) << H) <= N) ++H;
    for (int l = H - 1; l >= 0; --l) {
        const uint32_t lo = uint32_t(1) << l;
        const uint32_t hi = uint32_t(std::min<int64_t>((int64_t(1) << (l + 1)) - 1, N));
        hipLaunchKernelGGL(boxes_level, grid_for(hi - lo + 1), b, 0, st, d_pts, d_order, n, D, lo, hi, d_boxes);
        KD_HIP(hipGetLastError());
    }
    return KD_OK;
}

kd_status check_points_finite(const float* d_pts, int64_t N, int D, hipStream_t st, bool* ok) {
    *ok = true;
    if (N <= 0) return KD_OK;
    uint32_t* d_bad = nullptr;
    KD_HIP(hipMalloc(&d_bad, 4));
    hipError_t e = hipMemsetAsync(d_bad, 0, 4, st);
    const size_t n = size_t(N) * D;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(check_finite, dim3(unsigned(std::min<size_t>((n + 255) / 256, 4096))), dim3(256), 0, st,
                           d_pts, n, d_bad);
        e = hipGetLastError();
    }
    uint32_t bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_bad);
    if (e != hipSuccess) return hip_error(e, "kd_build: finiteness check");
    *ok = bad == 0;
    return KD_OK;
}

}  // namespace kd
