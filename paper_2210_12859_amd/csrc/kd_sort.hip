// kd_sort.hip -- Morton codes and a stable LSD radix sort of (code, index)
// pairs, used to reorder query batches along a Z-order curve so that queries
// that run together (in one wave, one CU, one XCD) traverse the same parts of
// the tree.  The reorder changes only the order in which queries are served,
// never any result.
//
// One sort pass over an 8-bit digit is three kernels:
//   radix_hist    per-tile digit counts            -> hist[digit][tile]
//   radix_scan    per-digit exclusive scan over tiles, in place, + digit totals
//   radix_scatter stable rank of every key inside its tile (wave ballots over
//                 the digit bits + LDS prefix over waves and rounds), then
//                 out[digit base + tile offset + rank]
// A tile is 256 threads x 16 rounds = 4096 keys; round r covers keys
// [r*256, (r+1)*256) of the tile, so tile order is preserved.
#include <hip/hip_runtime.h>

#include "kd_internal.h"

namespace kd {

namespace {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ROUNDS;

__device__ __forceinline__ uint32_t spread_bits(uint32_t v, int D) {
    // insert D-1 zero bits between the low bits of v
    if (D == 2) {
        v &= 0xffffu;
        v = (v | (v << 8)) & 0x00ff00ffu;
        v = (v | (v << 4)) & 0x0f0f0f0fu;
        v = (v | (v << 2)) & 0x33333333u;
        v = (v | (v << 1)) & 0x55555555u;
    } else if (D == 3) {
        v &= 0x3ffu;
        v = (v | (v << 16)) & 0x030000ffu;
        v = (v | (v << 8)) & 0x0300f00fu;
        v = (v | (v << 4)) & 0x030c30c3u;
        v = (v | (v << 2)) & 0x09249249u;
    } else {
        v &= 0xffu;
        v = (v | (v << 12)) & 0x000f000fu;
        v = (v | (v << 6)) & 0x03030303u;
        v = (v | (v << 3)) & 0x11111111u;
    }
    return v;
}

struct MortonArgs {
    const float* queries;
    uint32_t Q;
    int D;
    float lo[4];
    float scale[4];  // (2^bits) / extent, 0 for a flat axis
};

// 32-bit code, most significant spatial bit in bit 31 (D=3 uses bits 2..31).
__global__ void morton_codes(MortonArgs a, uint32_t* __restrict__ codes, uint32_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.Q) return;
    const int bits = a.D == 2 ? 16 : (a.D == 3 ? 10 : 8);
    const float maxc = float((1u << bits) - 1);
    uint32_t code = 0;
    for (int j = 0; j < a.D; ++j) {
        float u = (a.queries[size_t(i) * a.D + j] - a.lo[j]) * a.scale[j];
        u = u != u ? 0.0f : fminf(fmaxf(u, 0.0f), maxc);  // NaN -> 0, clamp
        code |= spread_bits(uint32_t(u), a.D) << (a.D - 1 - j);
    }
    if (a.D == 3) code <<= 2;
    codes[i] = code;
    vals[i] = i;
}

__global__ __launch_bounds__(SORT_THREADS) void radix_hist(const uint32_t* __restrict__ keys, uint32_t n,
                                                           int shift, uint32_t* __restrict__ hist,
                                                           uint32_t ntiles) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const uint32_t i = base + r * SORT_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[size_t(threadIdx.x) * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// One block per digit: exclusive scan of hist[digit][0..ntiles) in place;
// totals[digit] = sum.
__global__ __launch_bounds__(SORT_THREADS) void radix_scan(uint32_t* __restrict__ hist, uint32_t ntiles,
                                                           uint32_t* __restrict__ totals) {
    __shared__ uint32_t part[SORT_THREADS];
    uint32_t* row = hist + size_t(blockIdx.x) * ntiles;
    const uint32_t per = (ntiles + SORT_THREADS - 1) / SORT_THREADS;
    const uint32_t b = threadIdx.x * per;
    const uint32_t e = b + per < ntiles ? b + per : ntiles;
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i) s += row[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive scan of part (Hillis-Steele)
    for (int off = 1; off < SORT_THREADS; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (uint32_t i = b; i < e; ++i) {
        uint32_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (threadIdx.x == SORT_THREADS - 1) totals[blockIdx.x] = part[SORT_THREADS - 1];
}

__global__ __launch_bounds__(SORT_THREADS) void radix_scatter(const uint32_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin, uint32_t n,
                                                              int shift, const uint32_t* __restrict__ hist,
                                                              uint32_t ntiles, const uint32_t* __restrict__ totals,
                                                              uint32_t* __restrict__ kout,
                                                              uint32_t* __restrict__ vout) {
    __shared__ uint32_t base_d[256];      // digit base + this tile's offset, advanced per round
    __shared__ uint32_t wcnt[4][256];     // per-wave digit counts of the current round
    __shared__ uint32_t tmp[256];
    const int t = threadIdx.x;
    const int w = t >> 6;
    // exclusive scan of totals -> digit base
    tmp[t] = totals[t];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = t >= off ? tmp[t - off] : 0u;
        __syncthreads();
        tmp[t] += v;
        __syncthreads();
    }
    base_d[t] = (t ? tmp[t - 1] : 0u) + hist[size_t(t) * ntiles + blockIdx.x];
    for (int ww = 0; ww < 4; ++ww) wcnt[ww][t] = 0;
    __syncthreads();

    const uint32_t tile0 = blockIdx.x * SORT_TILE;
    const uint64_t lt_mask = (uint64_t(1) << (t & 63)) - 1;
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const uint32_t i = tile0 + r * SORT_THREADS + t;
        const bool valid = i < n;
        uint32_t key = 0, val = 0, d = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
            d = (key >> shift) & 0xffu;
        }
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = base_d[d] + rank;
            for (int ww = 0; ww < w; ++ww) off += wcnt[ww][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        base_d[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        wcnt[0][t] = 0;
        wcnt[1][t] = 0;
        wcnt[2][t] = 0;
        wcnt[3][t] = 0;
        __syncthreads();
    }
}

// Job of class slot i (jobs sorted by slot_base).
__device__ __forceinline__ int find_job(const BatchJob* jobs, int njobs, uint32_t i) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].slot_base <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// key = job index in the top jb bits, the job-local Morton code below
__global__ void batch_morton_codes(const BatchJob* __restrict__ jobs, int njobs, int D, int jb, uint32_t n,
                                   uint32_t* __restrict__ codes, uint32_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = find_job(jobs, njobs, i);
    const BatchJob& J = jobs[j];
    const uint32_t row = i - J.slot_base;
    const int bits = D == 2 ? 16 : (D == 3 ? 10 : 8);
    const float maxc = float((1u << bits) - 1);
    uint32_t code = 0;
    for (int d = 0; d < D; ++d) {
        float u = (J.queries[size_t(row) * D + d] - J.lo[d]) * J.scale[d];
        u = u != u ? 0.0f : fminf(fmaxf(u, 0.0f), maxc);
        code |= spread_bits(uint32_t(u), D) << (D - 1 - d);
    }
    if (D == 3) code <<= 2;
    codes[i] = jb > 0 ? (uint32_t(j) << (32 - jb)) | (code >> jb) : code;
    vals[i] = i;
}

// ---- counting sort on the top B <= 20 Morton bits, fused with the gather ----
// The order of queries inside one bucket does not matter (a query's result
// never depends on which lane serves it or when), so buckets are filled with
// atomics: zero -> count -> exclusive scan -> scatter the gathered record.

__global__ void bucket_zero(uint32_t* __restrict__ cnt, uint32_t nb, uint32_t* __restrict__ extra, uint32_t nextra) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) cnt[i] = 0;
    if (i < nextra) extra[i] = 0;
}

__global__ void bucket_count(MortonArgs a, int B, uint32_t* __restrict__ cnt, uint32_t* __restrict__ bucket) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.Q) return;
    const int bits = a.D == 2 ? 16 : (a.D == 3 ? 10 : 8);
    const float maxc = float((1u << bits) - 1);
    uint32_t code = 0;
    for (int j = 0; j < a.D; ++j) {
        float u = (a.queries[size_t(i) * a.D + j] - a.lo[j]) * a.scale[j];
        u = u != u ? 0.0f : fminf(fmaxf(u, 0.0f), maxc);
        code |= spread_bits(uint32_t(u), a.D) << (a.D - 1 - j);
    }
    if (a.D == 3) code <<= 2;
    const uint32_t b = code >> (32 - B);
    bucket[i] = b;
    atomicAdd(&cnt[b], 1u);
}

// exclusive scan of cnt[0..nb) in place (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void bucket_scan(uint32_t* __restrict__ cnt, uint32_t nb) {
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (nb + 1023) / 1024;
    const uint32_t b = t * per;
    const uint32_t e = b + per < nb ? b + per : nb;
    uint32_t sum = 0;
    for (uint32_t i = b; i < e; ++i) sum += cnt[i];
    part[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t ? part[t - 1] : 0u;
    for (uint32_t i = b; i < e; ++i) {
        const uint32_t v = cnt[i];
        cnt[i] = run;
        run += v;
    }
}

template <int D>
__global__ void bucket_scatter(const float* __restrict__ queries, uint32_t Q, const uint32_t* __restrict__ bucket,
                               uint32_t* __restrict__ cursor, NodeRec<D>* __restrict__ sq) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q) return;
    const uint32_t pos = atomicAdd(&cursor[bucket[i]], 1u);
    NodeRec<D> r;
#pragma unroll
    for (int j = 0; j < D; ++j) r.c[j] = queries[size_t(i) * D + j];
    r.idx = int32_t(i);
    sq[pos] = r;
}

}  // namespace

size_t bucket_scratch_bytes(int64_t Q, int B) {
    return (size_t(1) << B) * sizeof(uint32_t) + size_t(Q) * sizeof(uint32_t) + 256;
}

// Counting sort of the queries on the top B Morton bits (1 <= B <= 20); the
// scatter writes the gathered traversal-order records into sq.  Also zeroes
// `extra` (nextra words) on the way.
kd_status bucket_sort_gather(kd_tree t, const float* queries, int64_t Q, int B, void* ws, void* sq,
                             uint32_t* extra, uint32_t nextra, hipStream_t st) {
    const uint32_t n = uint32_t(Q);
    const uint32_t nb = 1u << B;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws);
    uint32_t* bucket = cnt + nb;
    MortonArgs a;
    a.queries = queries;
    a.Q = n;
    a.D = t->dim;
    const int bits = t->dim == 2 ? 16 : (t->dim == 3 ? 10 : 8);
    for (int j = 0; j < 4; ++j) {
        const float ext = t->hi[j] - t->lo[j];
        a.lo[j] = t->lo[j];
        a.scale[j] = (j < t->dim && ext > 0.0f) ? float(1u << bits) / ext : 0.0f;
    }
    const uint32_t nz = nb > nextra ? nb : nextra;
    hipLaunchKernelGGL(bucket_zero, dim3((nz + 255) / 256), dim3(256), 0, st, cnt, nb, extra, nextra);
    hipLaunchKernelGGL(bucket_count, dim3((n + 255) / 256), dim3(256), 0, st, a, B, cnt, bucket);
    hipLaunchKernelGGL(bucket_scan, dim3(1), dim3(1024), 0, st, cnt, nb);
    const dim3 g((n + 255) / 256), b(256);
    switch (t->dim) {
        case 2: hipLaunchKernelGGL(bucket_scatter<2>, g, b, 0, st, queries, n, bucket, cnt, (NodeRec<2>*)sq); break;
        case 3: hipLaunchKernelGGL(bucket_scatter<3>, g, b, 0, st, queries, n, bucket, cnt, (NodeRec<3>*)sq); break;
        default: hipLaunchKernelGGL(bucket_scatter<4>, g, b, 0, st, queries, n, bucket, cnt, (NodeRec<4>*)sq); break;
    }
    KD_HIP(hipGetLastError());
    return KD_OK;
}

size_t batch_sort_scratch_bytes(int64_t n) {
    const size_t ntiles = size_t((n + SORT_TILE - 1) / SORT_TILE);
    return 4 * size_t(n) * sizeof(uint32_t) + (256 * ntiles + 256) * sizeof(uint32_t) + 256;
}

kd_status batch_sort(const BatchJob* d_jobs, int njobs, int dim, uint32_t n, int sort_bits, void* ws,
                     hipStream_t st, const uint32_t** perm_out) {
    *perm_out = nullptr;
    if (n <= 1) return KD_OK;
    int jb = 0;
    while ((1 << jb) < njobs) ++jb;
    if (sort_bits <= 0) return KD_OK;  // class slots are already in job order
    const uint32_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    uint32_t* k0 = reinterpret_cast<uint32_t*>(ws);
    uint32_t* v0 = k0 + n;
    uint32_t* k1 = v0 + n;
    uint32_t* v1 = k1 + n;
    uint32_t* hist = v1 + n;
    uint32_t* totals = hist + size_t(256) * ntiles;
    hipLaunchKernelGGL(batch_morton_codes, dim3((n + 255) / 256), dim3(256), 0, st, d_jobs, njobs, dim, jb, n, k0, v0);
    KD_HIP(hipGetLastError());
    // the job bits must take part in the sort: sort on at least jb top bits
    int bits = sort_bits < jb ? ((jb + 7) / 8) * 8 : sort_bits;
    if (bits > 32) bits = 32;
    for (int p = 0; p < bits / 8; ++p) {
        const int shift = 32 - bits + 8 * p;
        hipLaunchKernelGGL(radix_hist, dim3(ntiles), dim3(SORT_THREADS), 0, st, k0, n, shift, hist, ntiles);
        hipLaunchKernelGGL(radix_scan, dim3(256), dim3(SORT_THREADS), 0, st, hist, ntiles, totals);
        hipLaunchKernelGGL(radix_scatter, dim3(ntiles), dim3(SORT_THREADS), 0, st, k0, v0, n, shift, hist, ntiles,
                           totals, k1, v1);
        KD_HIP(hipGetLastError());
        uint32_t* tk = k0; k0 = k1; k1 = tk;
        uint32_t* tv = v0; v0 = v1; v1 = tv;
    }
    *perm_out = v0;
    return KD_OK;
}

size_t sort_scratch_bytes(int64_t Q) {
    const size_t ntiles = size_t((Q + SORT_TILE - 1) / SORT_TILE);
    return 4 * size_t(Q) * sizeof(uint32_t) + (256 * ntiles + 256) * sizeof(uint32_t) + 256;
}

// Sorts query slots by Morton code (top sort_bits bits).  perm_out receives
// slot -> caller row.  ws must hold sort_scratch_bytes(Q).  When sort_bits == 0
// perm_out is not written and false is returned (identity order).
kd_status morton_sort(kd_tree t, const float* queries, int64_t Q, int sort_bits, void* ws, hipStream_t st,
                      const uint32_t** perm_out) {
    *perm_out = nullptr;
    if (sort_bits <= 0 || Q <= 1) return KD_OK;
    const uint32_t n = uint32_t(Q);
    const uint32_t ntiles = uint32_t((Q + SORT_TILE - 1) / SORT_TILE);
    uint32_t* k0 = reinterpret_cast<uint32_t*>(ws);
    uint32_t* v0 = k0 + Q;
    uint32_t* k1 = v0 + Q;
    uint32_t* v1 = k1 + Q;
    uint32_t* hist = v1 + Q;
    uint32_t* totals = hist + size_t(256) * ntiles;

    MortonArgs a;
    a.queries = queries;
    a.Q = n;
    a.D = t->dim;
    const int bits = t->dim == 2 ? 16 : (t->dim == 3 ? 10 : 8);
    for (int j = 0; j < 4; ++j) {
        const float ext = t->hi[j] - t->lo[j];
        a.lo[j] = t->lo[j];
        a.scale[j] = (j < t->dim && ext > 0.0f) ? float(1u << bits) / ext : 0.0f;
    }
    hipLaunchKernelGGL(morton_codes, dim3((n + 255) / 256), dim3(256), 0, st, a, k0, v0);
    KD_HIP(hipGetLastError());
    const int passes = sort_bits / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 32 - sort_bits + 8 * p;
        hipLaunchKernelGGL(radix_hist, dim3(ntiles), dim3(SORT_THREADS), 0, st, k0, n, shift, hist, ntiles);
        hipLaunchKernelGGL(radix_scan, dim3(256), dim3(SORT_THREADS), 0, st, hist, ntiles, totals);
        hipLaunchKernelGGL(radix_scatter, dim3(ntiles), dim3(SORT_THREADS), 0, st, k0, v0, n, shift, hist,
                           ntiles, totals, k1, v1);
        KD_HIP(hipGetLastError());
        uint32_t* tk = k0; k0 = k1; k1 = tk;
        uint32_t* tv = v0; v0 = v1; v1 = tv;
    }
    *perm_out = v0;
    return KD_OK;
}

}  // namespace kd
