/*
 * kd_oracle.c -- CPU oracle for exact fcp / kNN queries over a left-balanced,
 * complete k-d tree stored in level order.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP path.
 *
 * What it computes (readings of the paper are listed in the design notes):
 *
 *  - Tree layout: level order, root at 0, children of n at 2n+1 and 2n+2,
 *    parent (n+1)/2-1 (paper Sec. 3, assumption list; Sec. 3.2).  The split
 *    dimension is implicit per level: floor(log2(n+1)) mod D (Sec. 3,
 *    "splitDimOf"; the builder's choice, here round-robin by level).
 *  - Build: the canonical left-balanced tree.  At position i with point set S,
 *    S is ordered by (coordinate in i's split dimension, caller index) and the
 *    element of rank leftSize(|S|) is stored at i; the smaller ranks form the
 *    left subtree, the larger ranks the right subtree (Sec. 1 and Sec. 4: the
 *    tree is unique once ties are fixed).
 *  - Query: the ordered recursive traversal of Sec. 3.1 (the five-step form):
 *    empty subtree -> return; process the node (possibly shrinking the search
 *    radius); pick the close child by the side of the plane the query lies on
 *    (Sec. 3.2: close side is the right child iff signedDist > 0); traverse the
 *    close subtree; then traverse the far subtree if it still overlaps the
 *    query range.  The range test is taken in squared form, non-strict:
 *    fl(sd*sd) <= current worst squared distance.
 *  - Result: the k smallest (d2, index) keys among points with d2 <= R2,
 *    ascending; empty slots are (-1, +inf).  d2 is summed left to right in
 *    IEEE binary32 with no fused multiply-add (build with -ffp-contract=off).
 *  - Brute force: the plain definition above, O(N) per query.
 *  - Learned-radius rule: start from worst0 = min(R2, fl(r0*r0)) (r0 finite
 *    and >= 0, else R2); if fewer than k points were found and worst0 < R2,
 *    run again from R2.
 *  - Stored split dimensions (Sec. 3 leaves the split dimension to the
 *    builder and lets a node carry it; Sec. 4 names node types that store
 *    it): the "widest" rule picks, at each node, the dimension of largest
 *    extent of the node's point set, extent_j = fl32(max_j - min_j), the
 *    lowest j among equal extents; the rest of the build is unchanged (the
 *    same ranks, ordered by (coordinate in that dimension, index)).  The
 *    traversal then reads each node's dimension from dims[pos].
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SENT_IDX INT32_MAX

/* ---------------------------------------------------------------- helpers */

static int level_of(int64_t pos) { /* floor(log2(pos+1)) */
    int l = 0;
    uint64_t v = (uint64_t)pos + 1;
    while (v > 1) { v >>= 1; ++l; }
    return l;
}

/* Number of nodes in the left subtree of a left-balanced complete tree with
 * n nodes: the left subtree is complete; its last level holds the first
 * min(last, 2^(h-1)) nodes of the tree's last level. */
int64_t oracle_left_size(int64_t n) {
    if (n <= 1) return 0;
    int h = 0;
    while (((int64_t)1 << (h + 1)) <= n) ++h;          /* h = floor(log2 n) */
    int64_t last = n - (((int64_t)1 << h) - 1);          /* nodes on last level */
    int64_t half = (int64_t)1 << (h - 1);
    int64_t inner = half - 1;                            /* full levels of left subtree */
    return inner + (last < half ? last : half);
}

static float sqdist(const float* a, const float* b, int D) {
    float dx = a[0] - b[0];
    float s = dx * dx;
    for (int j = 1; j < D; ++j) {
        float t = a[j] - b[j];
        float t2 = t * t;
        s = s + t2;
    }
    return s;
}

/* lexicographic (d2, idx) order; NaN compares as never-less */
static int key_less(float ad, int32_t ai, float bd, int32_t bi) {
    return ad < bd || (ad == bd && ai < bi);
}

/* ------------------------------------------------------------------ build */

typedef struct {
    const float* P;
    int D;
    int dim;
} sort_ctx;

static __thread sort_ctx g_sort;

static int cmp_by_dim(const void* a, const void* b) {
    int32_t ia = *(const int32_t*)a, ib = *(const int32_t*)b;
    float fa = g_sort.P[(int64_t)ia * g_sort.D + g_sort.dim];
    float fb = g_sort.P[(int64_t)ib * g_sort.D + g_sort.dim];
    if (fa < fb) return -1;
    if (fa > fb) return 1;
    return (ia > ib) - (ia < ib);
}

/* Dimension of largest extent fl32(max - min) over the n >= 1 points S[0..n),
 * the lowest dimension among equal extents (the builder's choice of split
 * dimension, stored per node: Sec. 3 assumption list, Sec. 4). */
static int widest_dim(const float* P, int D, const int32_t* S, int64_t n) {
    int best = 0;
    float best_ext = -1.0f;
    for (int j = 0; j < D; ++j) {
        float mn = P[(int64_t)S[0] * D + j], mx = mn;
        for (int64_t i = 1; i < n; ++i) {
            float v = P[(int64_t)S[i] * D + j];
            if (v < mn) mn = v;
            if (v > mx) mx = v;
        }
        float ext = mx - mn;
        if (ext > best_ext) {
            best_ext = ext;
            best = j;
        }
    }
    return best;
}

static void build_rec(const float* P, int64_t N, int D, int rule, int32_t* S, int64_t n,
                      int64_t pos, int32_t* order, uint8_t* dims) {
    if (pos >= N) return; /* then n == 0 */
    int dim = rule == 1 ? widest_dim(P, D, S, n) : level_of(pos) % D;
    if (dims) dims[pos] = (uint8_t)dim;
    g_sort.P = P; g_sort.D = D; g_sort.dim = dim;
    qsort(S, (size_t)n, sizeof(int32_t), cmp_by_dim);
    int64_t m = oracle_left_size(n);
    order[pos] = S[m];
    build_rec(P, N, D, rule, S, m, 2 * pos + 1, order, dims);
    build_rec(P, N, D, rule, S + m + 1, n - m - 1, 2 * pos + 2, order, dims);
}

/* order[pos] = caller index of the point stored at level-order position pos;
 * dims[pos] (nullable) = its split dimension.  rule 0: floor(log2(pos+1))
 * mod D; rule 1: the widest extent of the node's point set.
 * Returns 0, or -1 on bad arguments / allocation failure. */
int oracle_build_rule(const float* P, int64_t N, int D, int rule, int32_t* order, uint8_t* dims) {
    if (N < 0 || D < 1 || D > 8 || rule < 0 || rule > 1) return -1;
    if (N == 0) return 0;
    int32_t* S = (int32_t*)malloc((size_t)N * sizeof(int32_t));
    if (!S) return -1;
    for (int64_t i = 0; i < N; ++i) S[i] = (int32_t)i;
    build_rec(P, N, D, rule, S, N, 0, order, dims);
    free(S);
    return 0;
}

int oracle_build(const float* P, int64_t N, int D, int32_t* order) {
    return oracle_build_rule(P, N, D, 0, order, NULL);
}

/* ------------------------------------------------------------------ query */

typedef struct {
    const float* P;
    const int32_t* order;
    int64_t N;
    int D;
    const float* q;
    int k;
    float* ld2;      /* k-list, ascending by (d2, idx) */
    int32_t* lidx;
    int64_t visited; /* processed nodes (first visits of existing nodes) */
    int32_t* seq;    /* optional: processed positions in order */
    int64_t seq_cap;
    const uint8_t* dims; /* stored split dimensions, or NULL (by level) */
} knn_ctx;

static void list_insert(knn_ctx* c, float d2, int32_t idx) {
    int k = c->k;
    if (!key_less(d2, idx, c->ld2[k - 1], c->lidx[k - 1])) return;
    int j = k - 1;
    while (j > 0 && key_less(d2, idx, c->ld2[j - 1], c->lidx[j - 1])) {
        c->ld2[j] = c->ld2[j - 1];
        c->lidx[j] = c->lidx[j - 1];
        --j;
    }
    c->ld2[j] = d2;
    c->lidx[j] = idx;
}

static void knn_rec(knn_ctx* c, int64_t pos) {
    if (pos >= c->N) return;                       /* empty subtree */
    int32_t pidx = c->order[pos];
    const float* p = c->P + (int64_t)pidx * c->D;
    float d2 = sqdist(c->q, p, c->D);               /* process the node */
    if (c->seq && c->visited < c->seq_cap) c->seq[c->visited] = (int32_t)pos;
    c->visited++;
    list_insert(c, d2, pidx);
    int dim = c->dims ? c->dims[pos] : level_of(pos) % c->D;
    float sd = c->q[dim] - p[dim];
    int64_t close_c = sd > 0.0f ? 2 * pos + 2 : 2 * pos + 1;
    int64_t far_c = sd > 0.0f ? 2 * pos + 1 : 2 * pos + 2;
    knn_rec(c, close_c);
    float sd2 = sd * sd;
    if (sd2 <= c->ld2[c->k - 1]) knn_rec(c, far_c);
}

/* One kNN query from initial worst squared radius worst0 over a tree with
 * stored split dimensions dims[N] (NULL: by level).  Writes k entries.
 * Returns the number of non-empty entries (found). */
int oracle_knn_one_dims(const float* P, const int32_t* order, const uint8_t* dims, int64_t N, int D,
                        const float* q, int k, float worst0, int32_t* out_idx,
                        float* out_d2, int64_t* visited, int32_t* seq, int64_t seq_cap) {
    float* ld2 = (float*)malloc((size_t)k * sizeof(float));
    int32_t* lidx = (int32_t*)malloc((size_t)k * sizeof(int32_t));
    for (int j = 0; j < k; ++j) { ld2[j] = worst0; lidx[j] = SENT_IDX; }
    knn_ctx c = {P, order, N, D, q, k, ld2, lidx, 0, seq, seq_cap, dims};
    knn_rec(&c, 0);
    int found = 0;
    for (int j = 0; j < k; ++j) {
        if (lidx[j] == SENT_IDX) {
            out_idx[j] = -1;
            if (out_d2) out_d2[j] = INFINITY;
        } else {
            out_idx[j] = lidx[j];
            if (out_d2) out_d2[j] = ld2[j];
            ++found;
        }
    }
    if (visited) *visited = c.visited;
    free(ld2);
    free(lidx);
    return found;
}

int oracle_knn_one(const float* P, const int32_t* order, int64_t N, int D,
                   const float* q, int k, float worst0, int32_t* out_idx,
                   float* out_d2, int64_t* visited, int32_t* seq, int64_t seq_cap) {
    return oracle_knn_one_dims(P, order, NULL, N, D, q, k, worst0, out_idx, out_d2, visited, seq, seq_cap);
}

/* worst0 for a predicted radius r0 (learned-radius rule). */
float oracle_worst0(float R2, float r0) {
    if (!isfinite(r0) || r0 < 0.0f) return R2;
    float r2 = r0 * r0;
    return r2 < R2 ? r2 : R2;
}

/* Learned-radius query: exact, with fallback.  *fell_back = 1 when the second
 * pass from R2 ran.  visited sums both passes. */
int oracle_knn_learned_one(const float* P, const int32_t* order, int64_t N, int D,
                           const float* q, int k, float R2, float r0, int32_t* out_idx,
                           float* out_d2, int64_t* visited, int* fell_back) {
    float w0 = oracle_worst0(R2, r0);
    int64_t v1 = 0, v2 = 0;
    int found = oracle_knn_one(P, order, N, D, q, k, w0, out_idx, out_d2, &v1, NULL, 0);
    *fell_back = 0;
    if (found < k && w0 < R2) {
        found = oracle_knn_one(P, order, N, D, q, k, R2, out_idx, out_d2, &v2, NULL, 0);
        *fell_back = 1;
    }
    if (visited) *visited = v1 + v2;
    return found;
}

/* ------------------------------------------------------------ brute force */

/* The plain definition: all points with d2 <= R2, the k smallest by
 * (d2, caller index), ascending; empty slots (-1, +inf). */
void oracle_brute_one(const float* P, int64_t N, int D, const float* q, int k, float R2,
                      int32_t* out_idx, float* out_d2) {
    float* ld2 = (float*)malloc((size_t)k * sizeof(float));
    int32_t* lidx = (int32_t*)malloc((size_t)k * sizeof(int32_t));
    int cnt = 0;
    for (int64_t i = 0; i < N; ++i) {
        float d2 = sqdist(q, P + i * D, D);
        if (!(d2 <= R2)) continue;
        /* insert into the first cnt entries kept ascending, capped at k */
        if (cnt == k && !key_less(d2, (int32_t)i, ld2[k - 1], lidx[k - 1])) continue;
        int j = cnt < k ? cnt : k - 1;
        if (cnt < k) ++cnt;
        while (j > 0 && key_less(d2, (int32_t)i, ld2[j - 1], lidx[j - 1])) {
            ld2[j] = ld2[j - 1];
            lidx[j] = lidx[j - 1];
            --j;
        }
        ld2[j] = d2;
        lidx[j] = (int32_t)i;
    }
    for (int j = 0; j < k; ++j) {
        out_idx[j] = j < cnt ? lidx[j] : -1;
        if (out_d2) out_d2[j] = j < cnt ? ld2[j] : INFINITY;
    }
    free(ld2);
    free(lidx);
}

/* -------------------------------------------------- range queries (brute) */

/* All points within the radius (Sec. 3 names sphere and box query primitives
 * and un-ordered traversals as variants of the method; d2 <= R2 as defined
 * above):
 * returns their number; the k smallest of them by (d2, caller index) go to
 * out_idx / out_d2 as in oracle_brute_one (k = 0: count only). */
int64_t oracle_radius_one(const float* P, int64_t N, int D, const float* q, float R2, int k,
                          int32_t* out_idx, float* out_d2) {
    int64_t count = 0;
    for (int64_t i = 0; i < N; ++i)
        if (sqdist(q, P + i * D, D) <= R2) ++count;
    if (k > 0) oracle_brute_one(P, N, D, q, k, R2, out_idx, out_d2);
    return count;
}

/* All points inside the axis-aligned box [lo, hi] (Sec. 3: a box as the
 * query primitive; lo[j] <= p[j] <= hi[j] in every dimension, inclusive):
 * returns their number; the k smallest caller
 * indices of them, ascending, go to out_idx, -1 after them (k = 0: count
 * only).  Scanning indices upwards, the first k found are the smallest. */
int64_t oracle_box_one(const float* P, int64_t N, int D, const float* lo, const float* hi, int k,
                       int32_t* out_idx) {
    int64_t count = 0;
    for (int64_t i = 0; i < N; ++i) {
        int in = 1;
        for (int j = 0; j < D; ++j)
            if (!(lo[j] <= P[i * D + j] && P[i * D + j] <= hi[j])) in = 0;
        if (!in) continue;
        if (count < k) out_idx[count] = (int32_t)i;
        ++count;
    }
    for (int64_t j = count; j < k; ++j) out_idx[j] = -1;
    return count;
}

/* ------------------------------------------------- threaded batch drivers */

typedef struct {
    int mode; /* 0 tree, 1 brute, 2 learned, 3 radius, 4 box */
    const float* P;
    const int32_t* order;
    int64_t N;
    int D;
    const float* Qp;
    int64_t Q;
    int k;
    float R2;
    const float* r0;
    int32_t* out_idx;
    float* out_d2;
    int64_t* visited;
    int32_t* fell_back;
    int64_t next;       /* shared chunk cursor */
    pthread_mutex_t mu;
    int64_t* count;     /* radius / box: points found per query */
    const uint8_t* dims; /* tree mode: stored split dimensions, or NULL */
} batch_job;

#define CHUNK 4096

static void* batch_worker(void* arg) {
    batch_job* b = (batch_job*)arg;
    for (;;) {
        pthread_mutex_lock(&b->mu);
        int64_t lo = b->next;
        b->next += CHUNK;
        pthread_mutex_unlock(&b->mu);
        if (lo >= b->Q) break;
        int64_t hi = lo + CHUNK < b->Q ? lo + CHUNK : b->Q;
        for (int64_t i = lo; i < hi; ++i) {
            if (b->mode == 3 || b->mode == 4) {
                /* radius: queries [Q][D]; box: [Q][2][D] (low corner, high corner) */
                int32_t* oi = b->out_idx ? b->out_idx + i * b->k : NULL;
                float* od = b->out_d2 ? b->out_d2 + i * b->k : NULL;
                if (b->mode == 3)
                    b->count[i] = oracle_radius_one(b->P, b->N, b->D, b->Qp + i * b->D, b->R2, b->k, oi, od);
                else
                    b->count[i] = oracle_box_one(b->P, b->N, b->D, b->Qp + i * 2 * b->D,
                                                 b->Qp + i * 2 * b->D + b->D, b->k, oi);
                continue;
            }
            const float* q = b->Qp + i * b->D;
            int32_t* oi = b->out_idx + i * b->k;
            float* od = b->out_d2 ? b->out_d2 + i * b->k : NULL;
            int64_t v = 0;
            if (b->mode == 0) {
                oracle_knn_one_dims(b->P, b->order, b->dims, b->N, b->D, q, b->k, b->R2, oi, od, &v, NULL, 0);
            } else if (b->mode == 1) {
                oracle_brute_one(b->P, b->N, b->D, q, b->k, b->R2, oi, od);
            } else {
                int fb = 0;
                oracle_knn_learned_one(b->P, b->order, b->N, b->D, q, b->k, b->R2, b->r0[i],
                                       oi, od, &v, &fb);
                if (b->fell_back) b->fell_back[i] = fb;
            }
            if (b->visited) b->visited[i] = v;
        }
    }
    return NULL;
}

static int run_batch(batch_job* b, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    b->next = 0;
    pthread_mutex_init(&b->mu, NULL);
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, batch_worker, b) != 0) break;
        ++started;
    }
    batch_worker(b);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&b->mu);
    return 0;
}

/* Q queries ([Q][D] row-major) through the recursive traversal.
 * out_idx / out_d2 are [Q][k]; visited (nullable) is [Q]. */
int oracle_knn_batch(const float* P, const int32_t* order, int64_t N, int D,
                     const float* queries, int64_t Q, int k, float R2, int32_t* out_idx,
                     float* out_d2, int64_t* visited, int nthreads) {
    if (k < 1 || N < 0 || Q < 0) return -1;
    batch_job b = {0, P, order, N, D, queries, Q, k, R2, NULL, out_idx, out_d2, visited, NULL};
    return run_batch(&b, nthreads);
}

/* The same over a tree with stored split dimensions dims[N]. */
int oracle_knn_batch_dims(const float* P, const int32_t* order, const uint8_t* dims, int64_t N, int D,
                          const float* queries, int64_t Q, int k, float R2, int32_t* out_idx,
                          float* out_d2, int64_t* visited, int nthreads) {
    if (k < 1 || N < 0 || Q < 0) return -1;
    batch_job b = {0, P, order, N, D, queries, Q, k, R2, NULL, out_idx, out_d2, visited, NULL};
    b.dims = dims;
    return run_batch(&b, nthreads);
}

int oracle_brute_batch(const float* P, int64_t N, int D, const float* queries, int64_t Q,
                       int k, float R2, int32_t* out_idx, float* out_d2, int nthreads) {
    if (k < 1 || N < 0 || Q < 0) return -1;
    batch_job b = {1, P, NULL, N, D, queries, Q, k, R2, NULL, out_idx, out_d2, NULL, NULL};
    return run_batch(&b, nthreads);
}

int oracle_knn_learned_batch(const float* P, const int32_t* order, int64_t N, int D,
                             const float* queries, int64_t Q, int k, float R2,
                             const float* r0, int32_t* out_idx, float* out_d2,
                             int64_t* visited, int32_t* fell_back, int nthreads) {
    if (k < 1 || N < 0 || Q < 0) return -1;
    batch_job b = {2, P, order, N, D, queries, Q, k, R2, r0, out_idx, out_d2, visited, fell_back};
    return run_batch(&b, nthreads);
}

int oracle_radius_batch(const float* P, int64_t N, int D, const float* queries, int64_t Q, int k, float R2,
                        int32_t* out_idx, float* out_d2, int64_t* count, int nthreads) {
    if (k < 0 || N < 0 || Q < 0) return -1;
    batch_job b = {3, P, NULL, N, D, queries, Q, k, R2, NULL, out_idx, out_d2, NULL, NULL};
    b.count = count;
    return run_batch(&b, nthreads);
}

int oracle_box_batch(const float* P, int64_t N, int D, const float* boxes, int64_t Q, int k, int32_t* out_idx,
                     int64_t* count, int nthreads) {
    if (k < 0 || N < 0 || Q < 0) return -1;
    batch_job b = {4, P, NULL, N, D, boxes, Q, k, 0.0f, NULL, out_idx, NULL, NULL, NULL};
    b.count = count;
    return run_batch(&b, nthreads);
}
