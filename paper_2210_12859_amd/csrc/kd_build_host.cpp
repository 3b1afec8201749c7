// kd_build_host.cpp -- host builder of the canonical left-balanced k-d tree.
//
// The tree is the level-order array of the paper's Sec. 3 assumption list
// (children of n at 2n+1 and 2n+2).  The split dimension of position n is
// floor(log2(n+1)) mod D.  A subtree with point set S stores at its root the
// element whose rank in S, ordered by (split coordinate, caller index), equals
// the size of the left subtree of a complete tree with |S| nodes; the smaller
// elements go left and the larger ones right.  With ties broken by the caller
// index the result is unique, so every correct builder produces the same
// array (Sec. 4).
//
// Partitioning uses std::nth_element on a permutation array (expected O(n)
// per level, O(N log N) total); the top levels fan out over std::threads.
#include <algorithm>
#include <thread>
#include <vector>

#include "kd_internal.h"

namespace kd {

int64_t left_subtree_size(int64_t n) {
    if (n < 2) return 0;
    int levels = 64 - __builtin_clzll((unsigned long long)n);  // levels of an n-node complete tree
    int64_t above_last = (int64_t(1) << (levels - 1)) - 1;      // nodes above the last level
    int64_t on_last = n - above_last;
    int64_t left_cap = int64_t(1) << (levels - 2);              // last-level slots under the left child
    return (above_last - 1) / 2 + std::min(on_last, left_cap);
}

namespace {

struct Builder {
    const float* pts;
    int dim;
    int64_t N;
    int32_t* perm;
    int32_t* order;

    static int level_of(int64_t pos) { return 63 - __builtin_clzll((unsigned long long)(pos + 1)); }

    void run(int64_t pos, int64_t lo, int64_t hi, int spawn_depth) {
        while (pos < N) {
            const int d = level_of(pos) % dim;
            const int64_t m = left_subtree_size(hi - lo);
            const float* p = pts;
            const int D = dim;
            std::nth_element(perm + lo, perm + lo + m, perm + hi, [p, D, d](int32_t a, int32_t b) {
                float fa = p[int64_t(a) * D + d], fb = p[int64_t(b) * D + d];
                return fa < fb || (fa == fb && a < b);
            });
            order[pos] = perm[lo + m];
            const int64_t mid = lo + m;
            if (spawn_depth > 0 && (hi - lo) > 65536) {
                std::thread th([this, pos, lo, mid, spawn_depth] { run(2 * pos + 1, lo, mid, spawn_depth - 1); });
                run(2 * pos + 2, mid + 1, hi, spawn_depth - 1);
                th.join();
                return;
            }
            run(2 * pos + 1, lo, mid, 0);
            pos = 2 * pos + 2;  // tail-iterate on the right subtree
            lo = mid + 1;
        }
    }
};

}  // namespace

void build_level_order(const float* pts, int64_t N, int dim, int32_t* order, int threads) {
    if (N <= 0) return;
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    std::vector<int32_t> perm(N);
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    int depth = 0;
    while ((1 << depth) < threads && depth < 6) ++depth;
    Builder b{pts, dim, N, perm.data(), order};
    b.run(0, 0, N, depth);
}

}  // namespace kd
