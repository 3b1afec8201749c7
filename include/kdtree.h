/*
 * kdtree.h -- C ABI of libkdtree.so: exact find-closest-point (fcp) and
 * k-nearest-neighbour (kNN) queries over left-balanced, complete k-d trees
 * stored in level order, traversed on an AMD Instinct MI355X (gfx950) with
 * the stack-free two-integer state machine of Wald, "A Stack-Free Traversal
 * Algorithm for Left-Balanced k-d Trees" (arXiv 2210.12859), Sec. 3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named points / queries / out_* / r0 / visited are DEVICE
 *    pointers (hipMalloc'd or torch CUDA tensors) unless stated otherwise.
 *    points and queries are float32, row-major [n][dim].
 *  - Results are int32 caller indices (0..N-1 of the points passed to
 *    kd_build, never tree positions) and float32 squared distances, [Q][k]
 *    row-major in the caller's query order, each row ascending by the key
 *    (d2, index).  Empty slots hold index -1 and d2 = +inf.
 *  - Squared distances are IEEE binary32: d2 = ((dx0*dx0 + dx1*dx1) + ...)
 *    with dx_j = q_j - p_j, left to right, no fused multiply-add, no
 *    flush-to-zero.  A point is eligible when d2 <= fl32(maxRadius*maxRadius)
 *    (inclusive; maxRadius = +inf means unbounded).  Ties in d2 go to the
 *    smaller point index.
 *  - stream is a hipStream_t passed as void* (NULL = the default stream).
 *    Query calls are asynchronous on it; the caller keeps every pointer alive
 *    and unmodified until the stream has reached the call.
 *  - Errors: every call returns a kd_status.  Arguments are validated before
 *    anything is enqueued; on error no output is touched.  kd_last_error()
 *    gives a thread-local message for the last non-OK status.  A device fault
 *    of an earlier asynchronous call surfaces as KD_EHIP from a later call.
 *  - Trees and models are immutable after creation; concurrent queries on
 *    different streams against one tree are safe.
 */
#ifndef KDTREE_H
#define KDTREE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kd_tree_s* kd_tree;   /* opaque, owned by the library */
typedef struct kd_model_s* kd_model; /* opaque, owned by the library */
typedef void* kd_stream;             /* a hipStream_t */

typedef enum {
    KD_OK = 0,
    KD_EINVAL = -1,       /* bad argument; nothing enqueued */
    KD_ENOMEM = -2,       /* device or host allocation failed */
    KD_EHIP = -3,         /* HIP runtime error (possibly from an earlier call) */
    KD_EUNSUPPORTED = -4  /* valid request this build does not implement */
} kd_status;

/* Largest supported k; k values other than 1,4,8,16,32,64 are served by the
 * next larger compiled list size, returning its first k entries (exact: the
 * k-best list is a prefix of any longer one). */
#define KD_MAX_K 64
/* Largest point count.  The traversal keeps 1-based node ids in int32: the
 * children of id i are 2i and 2i + 1 (the level-order children 2n+1, 2n+2 of
 * Sec. 3.2, shifted by one), so the largest id N and its child ids must stay
 * below 2^31: N <= 2^30 - 1. */
#define KD_MAX_POINTS ((1LL << 30) - 1)

/* Launch tuning.  Every setting gives byte-identical results; only speed
 * differs.  Passing NULL means "the options kd_autotune chose for this tree
 * and k, else the built-in defaults"; in a struct, a field at its "default"
 * value below takes the built-in default. */
typedef struct {
    int block;       /* threads per workgroup: 256, 512 or 1024 (k > 16: 256); 64, 128
                        also accepted; 0 = default (256) */
    int lds_levels;  /* top tree levels staged in each workgroup's LDS at launch
                        (node ids < 2^L, paper level order): steps at those
                        nodes read LDS instead of global memory.  0 or -1 =
                        none (default; measured no faster: the top levels stay
                        in L1/L2), 1..12, at most 64 KB of records (dim 4:
                        L <= 11).  kd_fcp / kd_knn / kd_knn_ex only; the
                        learned, batched and cooperative kernels read global
                        memory. */
    int sort_bits;   /* Morton bits the queries are sorted on before traversal:
                        0 keeps the caller's order; 1..32 is rounded up to a
                        whole byte (8, 16, 24, 32); -1 = default (16) */
    int waves_per_cu;/* persistent grid size in waves per compute unit (capped by
                        occupancy); 0 = default (32 for fcp / k = 1, else 24) */
    int heavy_trips; /* a query still unfinished after this many traversal loop
                        trips (checked every 16th trip of its wave, so up to 15
                        more) is handed to a second kernel in which a whole wave
                        finishes it (same results; keeps one far-off query from
                        holding the launch); -1 = never, 0 = default
                        (KD_DEFAULT_HEAVY_TRIPS, KD_DEFAULT_HEAVY_TRIPS_BOXES
                        with subtree boxes).  No hand-off happens when the
                        per-query visited count is requested, which is the
                        single-lane traversal's by definition. */
    int prune;       /* pruning rule (results are identical under both):
                        1 = split planes only, the paper's rule (the far child
                        is entered when the squared distance to its split
                        plane is <= the current k-th distance);
                        2 = that, and a subtree whose bounding box (of its
                        points, stored with the tree) lies farther than the
                        k-th distance is left on entry without processing any
                        of its nodes;
                        0 = default: 2, or 1 when the visited count is
                        requested. */
} kd_opts;

#define KD_DEFAULT_HEAVY_TRIPS 1024
/* default trip budget when subtree boxes prune (opts.prune 0 or 2): the box
 * test already shortens the long traversals the hand-off is for */
#define KD_DEFAULT_HEAVY_TRIPS_BOXES 4096

/* ------------------------------------------------------------ tree build */

/* Builds the canonical left-balanced, complete k-d tree over N points of
 * dimension dim (paper Sec. 1 and Sec. 3 assumption list): level-order array,
 * children of node n at 2n+1 and 2n+2, split dimension floor(log2(n+1)) mod
 * dim, and at every node the element of rank leftSize(|S|) of its subtree set
 * S ordered by (split coordinate, caller index) -- the unique tree once ties
 * are broken by index (Sec. 4 notes that any builder yields the same tree).
 *   points : device, float32 [N][dim]; read only.  NaN or +-inf -> KD_EINVAL.
 *   N      : 0 <= N <= KD_MAX_POINTS.  N = 0 gives an empty tree whose queries
 *            return all -1.
 *   dim    : 2, 3 or 4.
 *   out    : receives the tree; free with kd_tree_free.
 * Synchronises the stream (the build runs on the GPU; see kd_build_ex). */
kd_status kd_build(const float* points, int64_t N, int dim, kd_stream stream, kd_tree* out);

/* Split-dimension rules of kd_build_ex.  The paper leaves the split
 * dimension to the builder and lets a node carry it (Sec. 3, its assumption
 * list; Sec. 4, node types with a stored dimension).
 *   KD_SPLIT_LEVEL  : node at level l splits on l mod dim, nothing stored
 *                     (the tree of kd_build).
 *   KD_SPLIT_WIDEST : each node splits on the dimension of largest extent
 *                     fl32(max - min) of its subtree's points, the lowest
 *                     dimension on equal extents; the rest of the rule is
 *                     unchanged (rank leftSize, order by (coordinate in that
 *                     dimension, caller index)).  Stored as 2 bits per node
 *                     (one byte per node holding the node's and its three
 *                     nearest ancestors' dimensions). */
#define KD_SPLIT_LEVEL 0
#define KD_SPLIT_WIDEST 1

/* kd_build with a split-dimension rule.  Trees built with KD_SPLIT_WIDEST
 * are accepted by kd_fcp, kd_knn, kd_knn_ex (opts.lds_levels must be 0),
 * kd_knn_noalloc, kd_autotune, kd_radius_search and kd_box_search; the
 * learned-radius calls and batches return KD_EUNSUPPORTED for them.  Results
 * are the same exact kNN rows for either rule (the set of the k nearest by
 * (d2, index) does not depend on the tree); processed-node counts differ. */
kd_status kd_build_ex(const float* points, int64_t N, int dim, int split, kd_stream stream,
                      kd_tree* out);

/* Same, from a HOST float32 [N][dim] array (no device read of the input). */
kd_status kd_build_host(const float* host_points, int64_t N, int dim, kd_tree* out);

/* The same canonical level-order permutation computed on the host only (no
 * device involved): host_order[pos] = caller index of the point at tree
 * position pos.  host_points is HOST float32 [N][dim], 1 <= dim <= 8.
 * Used to build trees for other consumers and to check the builder. */
kd_status kd_build_order_host(const float* host_points, int64_t N, int dim, int32_t* host_order);

kd_status kd_tree_free(kd_tree t);

/* Tree facts.  Any out pointer may be NULL. */
kd_status kd_tree_info(kd_tree t, int64_t* N, int* dim, float* bbox_lo4, float* bbox_hi4);

/* Copies the level-order permutation to HOST memory: order[pos] = caller
 * index of the point at tree position pos; order has N entries. */
kd_status kd_tree_order(kd_tree t, int32_t* host_order);

/* The split dimension of every tree position to HOST memory (uint8 [N];
 * may be NULL) and the tree's rule (*split = KD_SPLIT_LEVEL or
 * KD_SPLIT_WIDEST; may be NULL). */
kd_status kd_tree_dims(kd_tree t, uint8_t* host_dims, int* split);

/* --------------------------------------------------------------- queries */

/* find-closest-point (paper Sec. 4, the fcp kernel) = kNN with k = 1.
 *   queries : device float32 [Q][dim];  Q >= 0.
 *   maxRadius : >= 0 or +inf; NaN or negative -> KD_EINVAL.
 *   out_idx : device int32 [Q];  out_d2 : device float32 [Q] or NULL. */
kd_status kd_fcp(kd_tree t, const float* queries, int64_t Q, float maxRadius,
                 int32_t* out_idx, float* out_d2, kd_stream stream);

/* k nearest neighbours (paper Sec. 4, the knn kernel, bounded or unbounded).
 *   k : 1 <= k <= KD_MAX_K.   out_idx : device int32 [Q][k];
 *   out_d2 : device float32 [Q][k] or NULL.  Other arguments as kd_fcp. */
kd_status kd_knn(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius,
                 int32_t* out_idx, float* out_d2, kd_stream stream);

/* kd_knn with launch options and an optional per-query count of entered
 * nodes (first visits of existing nodes).  Under the paper's pruning rule
 * (opts.prune 1, the default when visited is given) every entered node is
 * processed, so this is the paper's processNode count; under prune = 2 it
 * also counts subtrees left at their root by the bounding-box test.
 *   visited : device uint32 [Q] or NULL.   opts : may be NULL. */
kd_status kd_knn_ex(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius,
                    int32_t* out_idx, float* out_d2, uint32_t* visited,
                    const kd_opts* opts, kd_stream stream);

/* Device scratch of one query call.  kd_fcp, kd_knn, kd_knn_ex,
 * kd_knn_learned and kd_knn_with_radius use a per-stream workspace that the
 * library allocates on first use and keeps (growing it when a larger call
 * comes) until the process ends; this returns the bytes such a call of Q
 * queries needs, an upper bound over dim and launch options (query records,
 * sort buffers, work counters, hand-off rows).
 *   k     : validated (1..KD_MAX_K); the size does not depend on it.
 *   flags : 0, or KD_WS_LEARNED for the per-query initial radii of the
 *           learned-radius calls.
 *   bytes : host; receives the size (0 for Q = 0).
 * Host only: no device call, no allocation. */
#define KD_WS_LEARNED 1
kd_status kd_workspace_size(int64_t Q, int k, int flags, size_t* bytes);

/* kd_knn for callers that cannot allocate device memory: code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, validation, kernels and results as kd_knn (default launch
 * options, or the ones kd_autotune kept for the tree), but the call's scratch
 * comes from one fixed device array of KD_NOALLOC_SCRATCH_BYTES that the
 * library's code object holds on every device it runs on, from module load
 * until the process ends; the call itself allocates nothing and creates no
 * events (kd_timing_enable does not apply to it).  The caller still provides
 * queries and outputs.
 *   Capacity: the scratch a call needs is kd_workspace_size's per-dim figure;
 *   64 MiB holds Q <= 1,104,800 queries for dim 2 and 3 and Q <= 616,042 for
 *   dim 4.  A larger Q fails with KD_EINVAL before anything is enqueued.
 *   The tree must live on the current device (else KD_EINVAL).
 *   Every call on a device shares that device's array, which keeps the last
 *   call's contents (the call clears its own counters on the stream before
 *   use): calls that overlap in time on one device race and give undefined
 *   results, so issue them on one stream or order them with events. */
#define KD_NOALLOC_SCRATCH_BYTES (64u << 20)
kd_status kd_knn_noalloc(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius,
                         int32_t* out_idx, float* out_d2, kd_stream stream);

/* ---------------------------------------------------------- range queries */

/* All points within a radius of each query (Sec. 3: the same stack-free
 * traversal, un-ordered: children are taken left then right, each entered
 * only when the query ball reaches its side of the split plane).
 *   queries   : device float32 [Q][dim];  0 <= Q < 2^31.
 *   maxRadius : >= 0 or +inf (NaN or negative -> KD_EINVAL); a point is in
 *               range when its binary32 squared distance (summed left to
 *               right, no contraction) is <= fl32(maxRadius^2), as kd_knn.
 *   cap       : 0..KD_MAX_K results kept per query.
 *   out_count : device uint32 [Q]: the number of points in range.
 *   out_idx   : device int32 [Q][cap] (may be NULL when cap = 0): the cap
 *               nearest points in range, ascending by (d2, caller index),
 *               i.e. exactly kd_knn(k = cap, maxRadius)'s rows; -1 after
 *               the last.
 *   out_d2    : device float32 [Q][cap] or NULL; +inf after the last.
 *   visited   : device uint32 [Q] or NULL: nodes the traversal entered
 *               (first visits; a subtree left at its root by the box test
 *               counts its root only).
 *   flags     : 0: split planes only, the paper's un-ordered traversal
 *               (every point in range is processed).  KD_RANGE_BOXES: a
 *               subtree is also tested against its bounding box when
 *               entered: left at once when the box and the query region are
 *               disjoint and, with cap = 0, counted whole (without visiting
 *               it) when the box lies inside the region.  Both tests are
 *               exact in binary32 (counts and rows do not depend on the
 *               flag).  The box tests pay for count-only queries over
 *               regions holding thousands of points (clustered 1M points,
 *               ~10^4 per region: 1.8-2.0x); on small regions, and whenever
 *               rows are kept, they cost more than they save.
 * An empty tree gives counts 0.  A NaN query has no point in range.
 * Scratch: the per-stream workspace of the kd_knn family (query records and
 * sort buffers: at most kd_workspace_size(Q) for radius queries; box queries
 * add their centres, dim x 4 bytes per query); queries are taken in Morton
 * order.  Asynchronous on `stream`. */
#define KD_RANGE_BOXES 1
kd_status kd_radius_search(kd_tree t, const float* queries, int64_t Q, float maxRadius, int cap,
                           int32_t* out_idx, float* out_d2, uint32_t* out_count, uint32_t* visited,
                           int flags, kd_stream stream);

/* All points inside axis-aligned boxes (the un-ordered traversal of Sec. 3,
 * each child entered only when the box reaches its side of the split plane).
 *   boxes     : device float32 [Q][2][dim]: low corner then high corner; a
 *               point p is inside when lo[j] <= p[j] <= hi[j] for every j
 *               (inclusive; a box with lo[j] > hi[j] or a NaN bound holds
 *               nothing).
 *   cap       : 0..KD_MAX_K;  out_idx : device int32 [Q][cap]: the cap
 *               smallest caller indices inside, ascending, -1 after the last.
 *   out_count : device uint32 [Q]: the number of points inside.
 *   visited, flags : as kd_radius_search.
 * Boxes are taken in the Morton order of their centres (the per-stream
 * workspace holds the centres too).  Asynchronous on `stream`. */
kd_status kd_box_search(kd_tree t, const float* boxes, int64_t Q, int cap, int32_t* out_idx,
                        uint32_t* out_count, uint32_t* visited, int flags, kd_stream stream);

/* Every point in range of every query, as one variable-length result:
 * query q's points are out_idx[offsets[q] .. offsets[q + 1]), caller
 * indices in the order the traversal reaches them (deterministic for a given
 * tree and query).  Two traversals: counts (with subtree boxes when flags
 * has KD_RANGE_BOXES), an exclusive scan into offsets, then, when the total
 * fits capacity, the indices (split planes only).
 *   queries / boxes, maxRadius : as kd_radius_search / kd_box_search.
 *   offsets  : device int64 [Q + 1]; always written (offsets[Q] = total).
 *   out_idx  : device int32 [capacity], or NULL with capacity 0.
 *   capacity : >= 0.  When the total exceeds it, only offsets and *total
 *              are written (call again with a larger out_idx).
 *   total    : HOST int64: the number of points in range over all queries.
 * Synchronises the stream (the total is read back).  Beside the per-stream
 * workspace of the query calls, the library keeps a second per-stream buffer
 * for the counts (4 bytes per query, grown on demand, kept until exit). */
kd_status kd_radius_search_all(kd_tree t, const float* queries, int64_t Q, float maxRadius,
                               int64_t* offsets, int32_t* out_idx, int64_t capacity, int64_t* total,
                               int flags, kd_stream stream);
kd_status kd_box_search_all(kd_tree t, const float* boxes, int64_t Q, int64_t* offsets,
                            int32_t* out_idx, int64_t capacity, int64_t* total, int flags,
                            kd_stream stream);

/* ------------------------------------------------- learned initial radius */

/* A small MLP (3 -> 64 -> 64 -> 1, ReLU; bfloat16 operands, float32
 * accumulation, trained on the GPU) predicts y ~ ln(distance to the k-th
 * neighbour) for each query.  A learned query starts its traversal from the
 * squared radius worst0 = min(R2, fl32(r0 * r0)), r0 = exp(y + margin), in
 * place of R2 (the search radius of Sec. 3 may start at any value that
 * contains the answer).  A query that finds fewer than k points within
 * worst0 < R2 restarts, in the same lane, from R2.  Results are therefore
 * byte-identical to kd_knn for ANY model: the model changes speed only.
 * The model is 3-D (trees of dim 3). */

typedef struct {
    int epochs;            /* passes over the training queries (default 20) */
    int batch;             /* samples per Adam step, 64 .. 2^20 (default 8192) */
    float lr;              /* Adam learning rate (default 1e-3; betas 0.9, 0.999) */
    uint64_t seed;         /* weight init and shuffling (default 0) */
    int64_t holdout;       /* last rows of train_q held out to set the margin;
                              0 = min(Qt/10, 100000) */
    float margin_quantile; /* margin = this quantile of held-out (label - y),
                              0..1 (default 0.999: a restarted query runs twice,
                              late in the launch, so few restarts pay) */
} kd_train_opts;

typedef struct {
    int64_t queries;       /* queries in the call */
    int64_t fallbacks;     /* queries re-run from R2 */
    int64_t handed_off;    /* queries finished by the cooperative hand-off kernel */
    int64_t visited;       /* nodes entered by the single-lane traversal, both runs
                              of every query summed (nodes the hand-off kernel
                              processes are not counted); equals the sum of the
                              per-query visited counts when those are requested */
    float sort_ms;         /* GPU time of each stage, from hipEvents on the */
    float radius_ms;       /* stream: query reorder, initial radius (MLP), */
    float traverse_ms;     /* traversal, hand-off kernel (0 when there is none) */
    float handoff_ms;
} kd_stats;

/* Trains a radius model for k on the tree: labels are the k-th neighbour
 * distances of train_q (device float32 [Qt][3], 128 <= Qt < 2^31) from the
 * plain traversal; forward, backward and Adam run in the library's HIP
 * kernels.  Weights start He-normal (seeded), biases at zero except the
 * output bias, which starts at the mean training label.  opts may be NULL.
 * Synchronises the stream. */
kd_status kd_radius_model_train(kd_tree t, const float* train_q, int64_t Qt, int k, const kd_train_opts* opts,
                                kd_model* out, kd_stream stream);

/* kd_knn with the model's initial radius (see above).  The initial-radius
 * run starts below the root: descending from the root while the split plane
 * lies farther than the initial radius (fl(sd^2) > worst0), every skipped
 * node's point and far subtree are farther than worst0 as well, so the run
 * covers the subtree of the deepest node reached; the restart from R2 covers
 * the whole tree.  visited (nullable, device uint32 [Q]) counts processed
 * nodes of both runs; stats (nullable, HOST) receives the counts and stage
 * times above (radius_ms includes the start-node descent), which
 * synchronises the stream. */
kd_status kd_knn_learned(kd_tree t, kd_model m, const float* queries, int64_t Q, int k, float maxRadius,
                         int32_t* out_idx, float* out_d2, uint32_t* visited, kd_stats* stats, const kd_opts* opts,
                         kd_stream stream);

/* The same query with caller radii: r0 is device float32 [Q] in
 * caller order (any value: NaN, negative or +inf means "no initial radius").
 * fell_back (nullable, device uint8 [Q]) receives 1 for queries re-run from
 * R2, and 2 for queries handed to the cooperative kernel (opts.heavy_trips)
 * before their initial-radius run ended (they are finished from R2).  For
 * checking the exact-fallback rule with arbitrary radii. */
kd_status kd_knn_with_radius(kd_tree t, const float* r0, const float* queries, int64_t Q, int k, float maxRadius,
                             int32_t* out_idx, float* out_d2, uint32_t* visited, uint8_t* fell_back,
                             const kd_opts* opts, kd_stream stream);

/* Model facts; loss_curve (HOST, nullable) receives up to loss_cap per-epoch
 * mean training losses. */
kd_status kd_model_info(kd_model m, int* k, float* margin, float* holdout_rmse, int* n_epochs, float* loss_curve,
                        int loss_cap);
/* HOST copies of the 4481 float32 parameters (order W1[64][3], b1[64],
 * W2[64][64], b2[64], w3[64], b3) and the input normalisation (lo, 1/extent). */
kd_status kd_model_get_params(kd_model m, float* host_params, float* lo3, float* inv3);
/* A model from HOST parameters (same order), normalisation and margin. */
kd_status kd_model_create(const float* host_params, const float* lo3, const float* inv3, float margin, int k,
                          kd_model* out);
kd_status kd_model_save(kd_model m, const char* path);
kd_status kd_model_load(const char* path, kd_model* out);
kd_status kd_model_free(kd_model m);

/* Test hooks.  kd_mlp_predict: y (device float32 [n]) for device queries
 * [n][3].  kd_mlp_grad: mean-squared-error loss and its gradient (HOST
 * float32 [4481], parameter order) for device queries [n][3] and device
 * targets [n], n <= 2^20; synchronises the stream. */
kd_status kd_mlp_predict(kd_model m, const float* queries, int64_t n, float* y, kd_stream stream);
kd_status kd_mlp_grad(kd_model m, const float* queries, const float* targets, int64_t n, float* host_grad,
                      float* host_loss, kd_stream stream);
/* kd_mlp_worst0: the initial squared radius of the learned query path,
 * worst0 = min(R2, fl32(r0 * r0)) with r0 = exp(y + margin) (R2 when r0 is
 * not finite), R2 = fl32(maxRadius^2), for device queries [n][3], written to
 * device float32 worst0[n] in the queries' order by the same kernel the
 * learned query uses.  Synchronises the stream.
 * kd_mlp_train_step: one step of the trainer on n device (query, target)
 * rows: forward, backward, and one Adam update (betas 0.9, 0.999 and eps 1e-8
 * as float32; bias corrections 1 - beta^step) of the model's float32
 * parameters, which change in place -- not for a model that queries are
 * using.  host_m, host_v (HOST float32 [4481], in/out) are Adam's moments;
 * step >= 1 is Adam's step number; host_grad (HOST [4481], nullable)
 * receives the gradient the update used, host_loss (nullable) the batch loss;
 * kd_model_get_params returns the updated parameters.  n <= 2^20;
 * synchronises the stream. */
kd_status kd_mlp_worst0(kd_model m, const float* queries, int64_t n, float maxRadius, float* worst0,
                        kd_stream stream);
kd_status kd_mlp_train_step(kd_model m, const float* queries, const float* targets, int64_t n, int step, float lr,
                            float* host_m, float* host_v, float* host_grad, float* host_loss, kd_stream stream);

/* ---------------------------------------------------------------- batched */

/* Many independent trees and query sets in one call.  Jobs are grouped by
 * (dimension, list size); each group runs as ONE persistent traversal launch
 * in which every lane carries its own tree, after a Morton sort of the
 * group's queries (each job along its own tree's curve).  Queries still
 * unfinished after the trip budget (opts.heavy_trips) are finished by the
 * cooperative kernel, one wave each, as in kd_knn.  3-D jobs with a radius
 * model (the job's own, else the call's) start from the model's initial
 * radius and restart from R2 when it held fewer than k points, as in
 * kd_knn_learned.  Per job, results are exactly those of kd_knn on that job,
 * whatever the model and the options. */
typedef struct {
    kd_tree tree;
    const float* queries;  /* device [Q][dim] */
    int64_t Q;
    int k;                 /* 1..64 */
    float maxRadius;
    int32_t* out_idx;      /* device [Q][k] */
    float* out_d2;         /* device [Q][k] or NULL */
    kd_model model;        /* radius model for this job (3-D trees), or NULL */
} kd_job;

typedef struct kd_batch_s* kd_batch;

/* Validates the jobs, allocates the batch's scratch (owned by the batch) and
 * captures the whole pipeline into a hipGraph (on a private stream when
 * stream is NULL).  The job pointers and models are baked into the graph:
 * they must stay valid for the batch's lifetime.
 *   model : nullable; the radius model of 3-D jobs whose kd_job.model is NULL.
 *   opts  : nullable; block, waves_per_cu, sort_bits, heavy_trips and prune
 *           apply to every group (waves_per_cu 0: 32 for k = 1, else 24;
 *           sort_bits -1: 16 Morton bits below the group's job-index bits,
 *           rounded up to whole bytes). */
kd_status kd_batch_create(const kd_job* jobs, int n_jobs, kd_model model, const kd_opts* opts, kd_stream stream,
                          kd_batch* out);
/* Replays the captured graph on stream (asynchronous). */
kd_status kd_batch_run(kd_batch b, kd_stream stream);
/* Frees the batch; the caller must have synchronised every stream it ran on. */
kd_status kd_batch_free(kd_batch b);
/* create + run + synchronise + free. */
kd_status kd_knn_batched(const kd_job* jobs, int n_jobs, kd_model model, const kd_opts* opts, kd_stream stream);
/* Autotuner of the batched pipeline: for each (dimension, list size) group,
 * runs the group's pipeline with each candidate launch option (workgroup size
 * 256 / 512 x waves per CU 16 / 24 / 32 x sort key bits 16 / 24 / 32), reps
 * timed runs each, checks that every candidate writes the same outputs (a
 * 64-bit checksum of the group's result rows; a difference is KD_EHIP), keeps
 * the fastest per group and captures the graph again.  Overwrites the jobs'
 * outputs (with the same results).  class_opts (HOST, nullable, n_classes
 * entries on input) receives the options kept per group, in kd_batch_info's
 * order; *n_classes (nullable) the number of groups.  Synchronises. */
kd_status kd_batch_autotune(kd_batch b, int reps, kd_stream stream, kd_opts* class_opts, int* n_classes);
/* The groups of a batch (HOST arrays of cap entries, each nullable):
 * dimension, compiled list size, query count. */
kd_status kd_batch_info(kd_batch b, int* n_classes, int* class_dim, int* class_k, int64_t* class_queries, int cap);

/* --------------------------------------------------------------- autotune */

/* Times the candidate launch options (workgroup size 256/512/1024 x waves
 * per CU 8..32 x Morton sort bits 0/16/24/32 x pruning rule x LDS levels
 * 0/10) on a sample of queries (device float32 [Qs][dim]) with the given k
 * and maxRadius, keeps the fastest on the tree for k's list size, and
 * returns it (best_out, best_ms are HOST and nullable).  Results never depend
 * on the choice: every candidate's results are checked equal to the first's
 * (64-bit checksum of the result rows; a difference is KD_EHIP).
 * Synchronises the stream. */
kd_status kd_autotune(kd_tree t, const float* sample_q, int64_t Qs, int k, float maxRadius, kd_opts* best_out,
                      float* best_ms, kd_stream stream);
/* The options kept on the tree for k (KD_EINVAL if none), and setting them
 * (for example from a cache file). */
kd_status kd_tree_get_tuned(kd_tree t, int k, kd_opts* out);
kd_status kd_tree_set_tuned(kd_tree t, int k, const kd_opts* opts);

/* ------------------------------------------------------------ timing */

/* Kernel timing for benchmarks.  While enabled, every launch of the library's
 * traversal kernel ("traverse") and of its other stages is bracketed by
 * hipEvents recorded on the stream it runs on.  kd_timing_collect waits for
 * the recorded events of one kernel name, returns the summed elapsed time in
 * milliseconds and the launch count, and forgets that kernel's events. */
kd_status kd_timing_enable(int on);
kd_status kd_timing_collect(const char* kernel, double* total_ms, int64_t* launches);

/* ------------------------------------------------------------ status */

const char* kd_status_str(kd_status s);
const char* kd_last_error(void);
/* Library version string, e.g. "kdtree-gfx950 0.1". */
const char* kd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KDTREE_H */
