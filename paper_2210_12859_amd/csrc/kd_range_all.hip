// kd_range_all.hip -- every point in range of every query, as one
// variable-length result (offsets + indices), for the radius and box queries
// of the un-ordered traversal (Sec. 3 names spheres and boxes as query
// primitives of the same traversal).
//
// Two traversals: the first counts the points in range of each query (with
// subtree boxes on request, which may count whole subtrees), an exclusive
// scan turns the counts into offsets, and the second writes each query's
// points from its offset on, in the order the traversal reaches them (split
// planes only, so every point in range is visited).  The scan is three
// kernels: per-block scans of 4,096 counts, one workgroup scanning the block
// totals, and a pass adding them.  Counts and totals sit in the stream's
// second scratch buffer (kept by the library like the first).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "kd_internal.h"

namespace kd {

namespace {

constexpr int SCAN_T = 256;               // threads per block
constexpr int SCAN_E = 16;                // consecutive elements per thread
constexpr int SCAN_B = SCAN_T * SCAN_E;   // elements per block
constexpr int SCAN_W = SCAN_T / 64;       // waves per block

__device__ __forceinline__ int64_t shfl_up64(int64_t v, int d) {
    const uint32_t lo = __shfl_up(uint32_t(uint64_t(v)), d);
    const uint32_t hi = __shfl_up(uint32_t(uint64_t(v) >> 32), d);
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Exclusive prefix of v over the block's threads; *total receives the sum.
__device__ int64_t block_exclusive(int64_t v, int64_t* sh, int64_t* total) {
    const int lane = int(threadIdx.x & 63), wave = int(threadIdx.x >> 6);
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = shfl_up64(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int w = 0; w < SCAN_W; ++w) {
            const int64_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[SCAN_W] = run;
    }
    __syncthreads();
    const int64_t r = x - v + sh[wave];
    *total = sh[SCAN_W];
    __syncthreads();
    return r;
}

// out[i] = inclusive prefix of counts[0..i] within i's block; bsum[b] = the
// block's total.
__global__ __launch_bounds__(SCAN_T) void scan_local(const uint32_t* __restrict__ counts, int64_t n,
                                                    int64_t* __restrict__ out, int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[SCAN_W + 1];
    const int64_t first = int64_t(blockIdx.x) * SCAN_B + int64_t(threadIdx.x) * SCAN_E;
    int64_t v[SCAN_E];
    int64_t run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_E; ++i) {
        run += first + i < n ? int64_t(counts[first + i]) : 0;
        v[i] = run;
    }
    int64_t total;
    const int64_t pre = block_exclusive(run, sh, &total);
#pragma unroll
    for (int i = 0; i < SCAN_E; ++i)
        if (first + i < n) out[first + i] = pre + v[i];
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the nb block totals in place (one workgroup).
__global__ __launch_bounds__(SCAN_T) void scan_totals(int64_t* __restrict__ bsum, int64_t nb) {
    __shared__ int64_t sh[SCAN_W + 1];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_B) {
        const int64_t first = base + int64_t(threadIdx.x) * SCAN_E;
        int64_t v[SCAN_E];
        int64_t run = 0;
#pragma unroll
        for (int i = 0; i < SCAN_E; ++i) {
            v[i] = run;  // exclusive within the thread
            run += first + i < nb ? bsum[first + i] : 0;
        }
        int64_t total;
        const int64_t pre = block_exclusive(run, sh, &total);
#pragma unroll
        for (int i = 0; i < SCAN_E; ++i)
            if (first + i < nb) bsum[first + i] = carry + pre + v[i];
        carry += total;
        __syncthreads();
    }
}

// out[i] += the totals of the blocks before i's; offsets[0] = 0.
__global__ __launch_bounds__(SCAN_T) void scan_add(int64_t* __restrict__ offsets, int64_t n,
                                                  const int64_t* __restrict__ bsum) {
    const int64_t first = int64_t(blockIdx.x) * SCAN_B + int64_t(threadIdx.x) * SCAN_E;
    const int64_t add = bsum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_E; ++i)
        if (first + i < n) offsets[1 + first + i] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
}

kd_status range_all(kd_tree t, const float* in, int64_t Q, bool box, float maxRadius, int64_t* offsets,
                    int32_t* out_idx, int64_t capacity, int64_t* total, int flags, kd_stream stream,
                    const char* fn) {
    std::string f(fn);
    if (!total) return set_error(KD_EINVAL, f + ": total is NULL");
    if (Q < 0 || Q >= (int64_t(1) << 31)) return set_error(KD_EINVAL, f + ": Q out of range [0, 2^31)");
    if (flags & ~KD_RANGE_BOXES) return set_error(KD_EINVAL, f + ": unknown flags");
    if (!box && (std::isnan(maxRadius) || maxRadius < 0.0f))
        return set_error(KD_EINVAL, f + ": maxRadius must be >= 0 or +inf");
    if (capacity < 0) return set_error(KD_EINVAL, f + ": capacity must be >= 0");
    if (capacity > 0 && !out_idx) return set_error(KD_EINVAL, f + ": out_idx is NULL");
    if (!t) return set_error(KD_EINVAL, f + ": tree is NULL");
    if (!offsets) return set_error(KD_EINVAL, f + ": offsets is NULL");
    if (Q > 0 && !in) return set_error(KD_EINVAL, f + (box ? ": boxes is NULL" : ": queries is NULL"));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    *total = 0;
    if (Q == 0 || t->N == 0) {
        KD_HIP(hipMemsetAsync(offsets, 0, size_t(Q + 1) * sizeof(int64_t), st));
        KD_HIP(hipStreamSynchronize(st));
        return KD_OK;
    }
    const int64_t nb = (Q + SCAN_B - 1) / SCAN_B;
    // counts and block totals live across both traversals, which use the
    // stream's main scratch: the second per-stream buffer holds them
    const size_t cnt_b = (size_t(Q) * 4 + 255) & ~size_t(255);
    void* aux = nullptr;
    kd_status s = aux_scratch(stream, cnt_b + size_t(nb) * 8, &aux);
    if (s != KD_OK) return s;
    uint32_t* cnt = static_cast<uint32_t*>(aux);
    int64_t* bs = reinterpret_cast<int64_t*>(static_cast<char*>(aux) + cnt_b);
    const float R2 = box ? 0.0f : maxRadius * maxRadius;  // binary32 product; +inf stays +inf
    s = run_range(t, in, Q, box, R2, 0, nullptr, nullptr, cnt, nullptr, (flags & KD_RANGE_BOXES) == 0, stream);
    if (s != KD_OK) return s;
    hipLaunchKernelGGL(scan_local, dim3(unsigned(nb)), dim3(SCAN_T), 0, st, cnt, Q, offsets + 1, bs);
    KD_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(SCAN_T), 0, st, bs, nb);
    KD_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_add, dim3(unsigned(nb)), dim3(SCAN_T), 0, st, offsets, Q, bs);
    KD_HIP(hipGetLastError());
    int64_t tot = 0;
    KD_HIP(hipMemcpyAsync(&tot, offsets + Q, sizeof(tot), hipMemcpyDeviceToHost, st));
    KD_HIP(hipStreamSynchronize(st));
    *total = tot;
    if (tot == 0 || tot > capacity) return KD_OK;
    // the same traversal again, writing each query's points from its offset
    s = run_range(t, in, Q, box, R2, 0, nullptr, nullptr, cnt, nullptr, true, stream, offsets, out_idx);
    if (s != KD_OK) return s;
    KD_HIP(hipStreamSynchronize(st));
    return KD_OK;
}

}  // namespace

}  // namespace kd

using namespace kd;

extern "C" {

kd_status kd_radius_search_all(kd_tree t, const float* queries, int64_t Q, float maxRadius, int64_t* offsets,
                               int32_t* out_idx, int64_t capacity, int64_t* total, int flags, kd_stream stream) {
    return range_all(t, queries, Q, false, maxRadius, offsets, out_idx, capacity, total, flags, stream,
                     "kd_radius_search_all");
}

kd_status kd_box_search_all(kd_tree t, const float* boxes, int64_t Q, int64_t* offsets, int32_t* out_idx,
                            int64_t capacity, int64_t* total, int flags, kd_stream stream) {
    return range_all(t, boxes, Q, true, 0.0f, offsets, out_idx, capacity, total, flags, stream,
                     "kd_box_search_all");
}

}  // extern "C"
