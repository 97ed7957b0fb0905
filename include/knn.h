/*
 * knn.h -- exact k-nearest-neighbour search with a kd-tree on one MI355X
 * (gfx950), after Patwary et al., "PANDA: Extreme Scale Parallel K-Nearest
 * Neighbor on Distributed Architectures" (arXiv 1607.08220).
 *
 * The library builds the paper's local kd-tree (Section III-A) on the GPU and
 * answers batched k-NN queries with the traversal of Algorithm 1
 * (Section III-B/III-C).  Every call enqueues HIP kernels on the caller's
 * stream; all point, query and output pointers are DEVICE pointers.
 *
 * Result definition (shared by every entry point).  For a query q and points
 * x_0..x_{n-1} the distance is the FP32 squared Euclidean distance
 *     D(q, x) = fl(...fl(fl(t_0*t_0) + fl(t_1*t_1)) ... + fl(t_{d-1}*t_{d-1})),
 *     t_j = fl(q_j - x_j),
 * IEEE binary32 round-to-nearest-even, separate multiply and add, summed left
 * to right.  The candidates are the indices i with i != self and D < r2_max;
 * the answer is the k smallest keys (D, i) in ascending lexicographic order,
 * padded with (index -1, distance +inf) when fewer than k candidates exist.
 * This result does not depend on the shape of the tree.
 *
 * Return codes: KNN_OK (0) or a negative KNN_E* code; knn_last_error() gives
 * a message for the calling thread.  No exceptions cross this interface.
 */
#ifndef KNN_H
#define KNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KNN_OK 0
#define KNN_EINVAL -1   /* bad argument (null pointer, size or parameter out of range) */
#define KNN_ENOMEM -2   /* device or host allocation failed */
#define KNN_EDEVICE -3  /* a HIP call failed; knn_last_error() holds its message */
#define KNN_EDEPTH -4   /* the tree would be deeper than max_depth */
#define KNN_ENOTFINITE -5 /* an input coordinate is NaN or infinite (the build requires finite points) */

#define KNN_MAX_DIM 16  /* dimensions supported: 1..KNN_MAX_DIM */
#define KNN_MAX_K 64    /* neighbours per query: 1..KNN_MAX_K */

typedef struct knn_tree knn_tree; /* opaque; owns all device memory of one tree */
typedef struct knn_build_plan knn_build_plan; /* opaque; see knn_build_plan_create */

/* Construction parameters (Section III-A1).  Zero selects the default. */
typedef struct {
    int32_t leaf_size;      /* bucket size: nodes with more points are split (default 32) */
    int32_t max_depth;      /* deepest allowed leaf level, root = 0 (default 64) */
    int32_t subtree_points; /* nodes of at most this many points are finished by one
                               wavefront in LDS (default: derived from dim, at most 1024) */
    int32_t split_block_nodes; /* level passes of at most this many nodes choose each split
                                  with a workgroup, larger ones with one wavefront per node
                                  (default 256; -1: always a wavefront); a scheduling knob,
                                  the tree does not depend on it */
} knn_build_params;

#define KNN_QUERY_STATS 9

/* Query parameters.  Zero selects the default. */
typedef struct {
    int32_t order;  /* 0 (default): process queries grouped by the leaf that contains them
                       (the one-wavefront-per-query form always takes input order);
                       1: process queries in input order */
    int32_t leaf_batch; /* 1..64, 0 = default: a wavefront scans buckets once at least
                           leaf_batch of every 64 of its unfinished lanes (one per query)
                           hold one; a scheduling knob, the result does not depend on it */
    int64_t* stats; /* NULL, or a device pointer to KNN_QUERY_STATS int64 counters the
                       traversal adds to; slower, for measurement only.  Summed over
                       queries: 0 nodes entered from above, 1 leaves scanned, 2 points
                       scanned (the traversal counts of Section V-B2), 3 traversal
                       steps, 4 heap inserts; summed over wavefronts (64 queries):
                       5 traversal-loop iterations, 6 bucket-row batches, 7 leaf
                       rounds, 8 heap-insert executions */
    int32_t traversal; /* 0 (default): below 5 dimensions form 3 for batches of at most
                          16,384 queries, else 1 (2 in 4 dimensions from k = 16 with buckets
                          of 16 or more points); from 5
                          dimensions form 3 up to 4,096 queries, form 4 with 32 lanes up
                          to 32,768 (where k and the depth fit), else 2; 1: stack-free walk from the
                          query's home leaf (each node keeps its parent); 2: Algorithm 1's
                          explicit stack, kept in LDS (used when the tree's depth fits);
                          3: Algorithm 1's explicit stack with one wavefront per query
                          (used when the tree is at most 63 levels deep and stats is
                          NULL; for deep searches answered with few queries);
                          4: the same with a team of team_lanes lanes per query (used
                          when k <= team_lanes, the tree is at most team_lanes - 1
                          levels deep and stats is NULL, else as 0);
                          a scheduling knob, the result does not depend on it */
    int32_t team_lanes; /* traversal 4: lanes per query, 8, 16 or 32 (0 = 32) */
} knn_query_params;

typedef struct {
    int64_t n;            /* points */
    int32_t dim;
    int32_t leaf_size;
    int32_t depth;        /* deepest leaf level (root = 0) */
    int32_t subtree_points;
    int64_t nodes;        /* inner nodes + leaves */
    int64_t leaves;
    int64_t device_bytes; /* device memory held by the tree */
    int32_t trees;        /* 1, or the number of trees of a forest (knn_build_batch) */
    int32_t pad_;
} knn_tree_info_t;

/* Host copy of a tree (knn_tree_export).  The caller allocates every array
 * with the sizes from knn_tree_info (N = nodes, n, d = dim); NULL skips one.
 * Node 0 is the root.  Inner node v splits dimension dim[v] at split[v]:
 * points with x[dim] < split are in child left[v], the others in left[v] + 1.
 * Leaves have dim[v] = -1 and hold packed positions [start[v], start[v] +
 * count[v]).  start/count are also filled for inner nodes (their range). */
typedef struct {
    int32_t* dim;    /* [N] */
    float* split;    /* [N] */
    int32_t* left;   /* [N], -1 for leaves */
    int32_t* parent; /* [N], -1 for the root */
    int32_t* start;  /* [N] */
    int32_t* count;  /* [N] */
    float* lo;       /* [N * d] tight bounding box, row per node */
    float* hi;       /* [N * d] */
    int32_t* perm;   /* [n]  packed position -> original point index */
    float* packed;   /* [n * d] coordinates in packed (bucket-contiguous) order */
} knn_tree_host;

/*
 * knn_build -- construct the kd-tree of Section III-A over n points.
 *   points  device pointer, row-major [n, dim] FP32 (finite values)
 *   n       1 .. 2^30 (node ids are int32)
 *   dim     1 .. KNN_MAX_DIM
 *   leaf_size >= 1 (0 = default 32)
 *   stream  a hipStream_t (NULL = default stream)
 *   out     receives the new tree; the caller frees it with knn_tree_free
 * Each node is split along the dimension of maximum variance of a sample of
 * min(1024, count) of its points (Section III-A1, split dimension), at the
 * sample point whose count of node points below it is closest to half
 * (Section III-A1, split point; a histogram over the sorted sample), by a
 * stable partition (Section III-A ii/iii) until nodes hold at most leaf_size
 * points (Section III-A1, bucket size); buckets are stored contiguously
 * (Section III-A iv).  The tree copies what it needs: `points` may be reused
 * once the call returns.  The call synchronizes `stream` before returning.
 * Errors: KNN_EINVAL, KNN_ENOMEM, KNN_EDEVICE, KNN_EDEPTH, KNN_ENOTFINITE (a
 * coordinate is NaN or infinite: checked while the points are copied in,
 * before any split is computed); no tree is returned on error.
 */
int knn_build(const float* points, int64_t n, int32_t dim, int32_t leaf_size, void* stream,
              knn_tree** out);

/* knn_build with all construction parameters (p may be NULL for defaults). */
int knn_build_ex(const float* points, int64_t n, int32_t dim, const knn_build_params* p,
                 void* stream, knn_tree** out);

/*
 * knn_build_batch -- build many independent trees in one call: tree t is built
 * over rows offsets[t] .. offsets[t+1]-1 of `points`, exactly as knn_build_ex
 * would build it from those rows alone (same splits, buckets and boxes).  All
 * trees go through the same level passes and subtree kernels, so the launch
 * count does not grow with the number of trees.  The result is one forest
 * handle whose tree t has root node t; query it with knn_query_batch.
 *   points   device pointer [offsets[trees], dim] FP32, the trees' rows concatenated
 *   offsets  HOST pointer [trees + 1]: offsets[0] = 0, strictly increasing
 *   trees    >= 1; all points together at most 2^30
 * Neighbour indices are rows of the concatenated array.  Errors as knn_build_ex.
 */
int knn_build_batch(const float* points, const int64_t* offsets, int32_t trees, int32_t dim,
                    const knn_build_params* p, void* stream, knn_tree** out);

/*
 * Build plans -- the build of Section III-A (as knn_build_batch) for a fixed
 * point count and forest layout, split into a set-up call that allocates and
 * uploads everything once, and runs that only enqueue kernels.  A run
 * allocates nothing, copies nothing between host and device and never waits,
 * so a HIP graph can capture it (queries on the plan's tree may follow it in
 * the same graph) and replay it over new point values.  A successful run
 * builds exactly the tree knn_build_batch builds from the same points.
 *
 * knn_build_plan_create(n, dim, offsets, trees, p, stream, out)
 *   n, dim     as knn_build_ex
 *   offsets    HOST pointer [trees + 1] as knn_build_batch, with offsets[trees]
 *              = n; or NULL with trees = 1 (one tree over all n points).
 *              Read during the call only.
 *   p          as knn_build_ex, except max_depth 0 = the largest tree's balanced
 *              depth + 8.  max_depth bounds every run and is the depth the
 *              plan's tree reports (query kernels size their stacks by it).
 *   stream     carries the one-time uploads; the call waits for them
 *   out        receives the plan.  Errors: KNN_EINVAL, KNN_ENOMEM.
 * knn_build_plan_run(plan, points, stream)
 *   points     device pointer [n, dim] FP32 (same layout as knn_build_batch)
 *   Enqueued on stream and not waited for.  Runs of one plan must not
 *   overlap.  Input errors found on the device (a non-finite coordinate, a
 *   tree deeper than max_depth, more level passes than the plan holds) are
 *   recorded there; the tree then answers every query with index -1 in all
 *   k places until a run succeeds.
 * knn_build_plan_finish(plan, stream, tree)
 *   Waits for stream and returns the status of the latest run it carried:
 *   KNN_OK, KNN_ENOTFINITE, KNN_EDEPTH or KNN_EDEVICE.  *tree (if tree is not
 *   NULL) receives the plan's tree, with its node count updated.
 * knn_build_plan_tree(plan)
 *   The plan's tree, without waiting (to capture queries after a run).  It
 *   belongs to the plan (knn_tree_free refuses it), is the same handle for the
 *   plan's whole life, and holds the latest completed run's tree.
 * knn_build_plan_destroy(plan)
 *   Waits for the queries on the plan's tree and the latest run enqueued
 *   outside a capture, then frees all of the plan's device memory.  Graph
 *   launches are the caller's to wait for.  NULL is a no-op.
 */
int knn_build_plan_create(int64_t n, int32_t dim, const int64_t* offsets, int32_t trees,
                          const knn_build_params* p, void* stream, knn_build_plan** out);
int knn_build_plan_run(knn_build_plan* plan, const float* points, void* stream);
int knn_build_plan_finish(knn_build_plan* plan, void* stream, knn_tree** tree);
knn_tree* knn_build_plan_tree(knn_build_plan* plan);
int knn_build_plan_destroy(knn_build_plan* plan);

/*
 * knn_query -- the k nearest neighbours of m queries (Algorithm 1).
 *   t         a tree from knn_build (a forest from knn_build_batch is rejected)
 *   queries   device pointer, row-major [m, dim] FP32
 *   m         >= 0 (0 is a no-op)
 *   k         1 .. KNN_MAX_K (k > n pads)
 *   out_idx   device pointer [m, k] int32: original point indices
 *   out_dist2 device pointer [m, k] FP32: squared distances, ascending by (D, idx)
 * Work is enqueued on `stream` and not waited for; the tree must outlive it.
 * Concurrent queries on one tree (any streams) are allowed.
 * Errors: KNN_EINVAL, KNN_ENOMEM, KNN_EDEVICE.
 */
int knn_query(const knn_tree* t, const float* queries, int64_t m, int32_t k, int32_t* out_idx,
              float* out_dist2, void* stream);

/*
 * knn_query_ex -- knn_query with Algorithm 1's search radius and self exclusion.
 *   self_ids  device pointer [m] int32 or NULL; self_ids[i] >= 0 removes that one
 *             point index from query i's candidates (-1 = none)
 *   r2_max    squared search radius r^2: only D < r2_max qualify (+inf = none)
 *   p         query parameters or NULL
 */
int knn_query_ex(const knn_tree* t, const float* queries, int64_t m, int32_t k,
                 const int32_t* self_ids, float r2_max, const knn_query_params* p,
                 int32_t* out_idx, float* out_dist2, void* stream);

/*
 * knn_query_noalloc -- knn_query_ex that allocates nothing, for callers that
 * cannot allocate device memory: code being captured into a graph, tight
 * serving loops, harnesses that forbid allocation.  Same arguments, result
 * and errors as knn_query_ex.  Its workspace (the grouping of queries by home
 * leaf) is a static device array of KNN_NOALLOC_WORKSPACE_BYTES that each
 * device holds from the first call there until the process ends.
 *   Workspace a call needs: none with order 1 or when one wavefront answers
 *   each query (traversal 3, the default for batches of at most 16,384
 *   queries); otherwise 4 (N + ceil(N / 4096)) + 12 m bytes with
 *   N = floor(n / 2^s) + 1, s the smallest shift giving n / 2^s <= 2^22 (for
 *   n >= 2^22, N is about 2^22: up to about 5.5 M queries fit).  A call that
 *   needs more fails with KNN_EINVAL before anything is launched.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (the counters that must start at zero are cleared by a
 * kernel of each call): calls that overlap on one device (other streams or
 * threads) race and corrupt each other's results -- serialise them.
 * knn_tree_free does not wait for these calls; the caller does.
 */
#define KNN_NOALLOC_WORKSPACE_BYTES (80ll << 20)
int knn_query_noalloc(const knn_tree* t, const float* queries, int64_t m, int32_t k,
                      const int32_t* self_ids, float r2_max, const knn_query_params* p,
                      int32_t* out_idx, float* out_dist2, void* stream);

/*
 * knn_query_batch -- knn_query_ex on a forest: query i searches only tree
 * tree_ids[i] (device pointer [m] int32, each in [0, trees)).  All queries
 * run in one batch of launches whatever trees they address.  Indices are rows
 * of the concatenated points; self_ids use the same numbering.  The ids are
 * checked on the device: a query whose id is outside [0, trees) reads no
 * node, gets a row of padding (-1, +inf) and is counted; knn_tree_errors
 * returns KNN_EINVAL and the count.
 */
int knn_query_batch(const knn_tree* t, const float* queries, const int32_t* tree_ids,
                    int64_t m, int32_t k, const int32_t* self_ids, float r2_max,
                    const knn_query_params* p, int32_t* out_idx, float* out_dist2, void* stream);

/*
 * knn_query_radius -- knn_query_ex with one search radius per query: only
 * points with D < r2[i] qualify for query i.  This is Algorithm 1 with its
 * input r given per query, as in the remote step of the distributed query
 * (Section III-B, steps 2 and 4): a query arrives with r' = the k-th distance
 * found on its owner, and the search prunes everything at or beyond it.
 *   r2  device pointer [m] FP32 squared radii (+inf = none; a NaN or a value
 *       <= 0 admits no point)
 * Other arguments and errors as knn_query_ex.
 */
int knn_query_radius(const knn_tree* t, const float* queries, int64_t m, int32_t k,
                     const int32_t* self_ids, const float* r2, const knn_query_params* p,
                     int32_t* out_idx, float* out_dist2, void* stream);

/*
 * knn_merge -- the k nearest of two candidate lists per query (Section III-B,
 * step 5: the local and the remote neighbours are merged by distance).
 *   idx_a, dist2_a  device pointers [m, ka]: one list per query, ascending by
 *                   (D, idx), padded at the end with (idx -1, D +inf)
 *   idx_b, dist2_b  device pointers [m, kb], the same form
 *   out_idx, out_dist2  device pointers [m, k]: the k smallest (D, idx) keys
 *                   of both lists, ascending, padded with (-1, +inf); an entry
 *                   present in both lists (same D and idx) counts once
 * ka, kb, k: 1 .. KNN_MAX_K.  The output may not alias an input.  Work is
 * enqueued on `stream`.  Errors: KNN_EINVAL, KNN_EDEVICE.
 */
int knn_merge(const int32_t* idx_a, const float* dist2_a, int32_t ka, const int32_t* idx_b,
              const float* dist2_b, int32_t kb, int64_t m, int32_t k, int32_t* out_idx,
              float* out_dist2, void* stream);

/*
 * Serving: resident trees answer a stream of query requests with continuous
 * batching (the query batching of Section III-B, step 2, applied to a request
 * stream).  A server keeps the given trees (which the caller keeps alive)
 * and runs one worker thread: pending requests for the same tree, of any k,
 * are packed into one batch (each query keeps its own k), admitted when a
 * stream is free and the batch's device memory fits in the budget beside the
 * batches already in flight, so requests that arrive while others run join
 * the next batch and batches on different streams overlap.  Each query is
 * answered exactly as by knn_query_ex, so results do not depend on the mix.
 */
typedef struct knn_server knn_server;

/* Server parameters; zero selects the default. */
typedef struct {
    int64_t hbm_budget_bytes; /* device memory the batches in flight may hold (0 = 4 GiB; a
                                 batch larger than the budget still runs when nothing else is
                                 in flight) */
    int32_t streams;          /* concurrent batches, 1..64 (0 = 4) */
    int32_t slot_max_queries; /* 0 (default): every request forms batches; n > 0: requests
                                 of at most min(n, 16384) queries are answered by the tree's
                                 slot kernel instead -- a persistent launch whose wavefronts
                                 take each new request over while it runs and answer its
                                 queries one wavefront per query, the request with the fewest
                                 queries left first; a launch stops admitting after 20 ms and
                                 ends when idle (the worker relaunches it), so it never holds
                                 a hardware queue long */
    int32_t slot_workgroups_per_cu; /* a slot kernel's workgroups of four wavefronts per
                                       compute unit, 1..8 (0 = 1) */
    int32_t slot_idle_us;     /* a slot kernel with nothing to do ends after this many
                                 microseconds (0 = 2000) */
} knn_server_params;

/* trees: host array of ntrees (>= 1) single trees on one device (each at
 * most 63 levels deep); p may be NULL for the defaults. */
int knn_server_create_ex(const knn_tree* const* trees, int32_t ntrees, const knn_server_params* p,
                         knn_server** out);

/* knn_server_create_ex with the given budget and stream count (batches only). */
int knn_server_create(const knn_tree* const* trees, int32_t ntrees, int64_t hbm_budget_bytes,
                      int32_t streams, knn_server** out);

/* Queue one request: m (1 .. 2^18) queries (device pointer [m, dim]) against
 * tree `tree` with k neighbours, optional self ids (device [m] or NULL);
 * results go to the caller's device buffers out_idx/out_dist2 [m, k], which
 * must stay valid until knn_server_wait returns for the ticket.  Thread-safe. */
int knn_server_submit(knn_server* s, int32_t tree, const float* queries, int64_t m, int32_t k,
                      const int32_t* self_ids, int32_t* out_idx, float* out_dist2,
                      int64_t* ticket);

/* Block until the request is complete (its results are in its buffers);
 * latency_ms (may be NULL) receives the time from submit to completion as
 * seen by the worker.  Each ticket is waited for once. */
int knn_server_wait(knn_server* s, int64_t ticket, double* latency_ms);

/* Counters, out[KNN_SERVER_STATS]: 0 requests submitted, 1 batches
 * launched, 2 queries answered, 3 peak device bytes held by batches in
 * flight, 4 most requests in one batch, 5 most batches in flight at once,
 * 6 most distinct k in one batch, 7 requests admitted while earlier work was
 * on the device (a batch launched beside another, or a request posted to a
 * running slot kernel), 8 requests answered by slot kernels, 9 slot-kernel
 * launches. */
#define KNN_SERVER_STATS 10
int knn_server_stats(knn_server* s, int64_t* out);

/* Finish every queued request, stop the worker and free the server (not the
 * trees).  NULL is OK. */
int knn_server_destroy(knn_server* s);

/*
 * knn_classify -- k-NN classification of each query by a majority vote of its
 * neighbours' labels, the baseline method the paper applies to its labelled
 * data (Section V-C).
 *   idx        device [m, k] int32 neighbour lists from a query, ascending by
 *              distance, -1 padding; every index < the number of labels
 *   labels     device int32 label of every point
 *   out_class  device [m] int32: the label with the most votes; between labels
 *              with equally many, the one whose first neighbour is nearer;
 *              -1 when the query has no neighbour
 *   out_votes  device [m] int32 or NULL: that label's vote count
 * Errors: KNN_EINVAL, KNN_EDEVICE.
 */
int knn_classify(const int32_t* idx, int64_t m, int32_t k, const int32_t* labels,
                 int32_t* out_class, int32_t* out_votes, void* stream);

/*
 * knn_regress -- k-NN regression (Section I names classification and
 * regression): the mean of the neighbours' values, summed in FP32 left to
 * right in neighbour order and divided by the neighbour count; NaN when the
 * query has no neighbour.  idx as in knn_classify; values device FP32 per
 * point; out device [m] FP32.
 */
int knn_regress(const int32_t* idx, int64_t m, int32_t k, const float* values, float* out,
                void* stream);

/* Free a tree and its device memory.  Waits for the latest query enqueued on
 * each stream that queried the tree (not for other work on the device), then
 * returns the memory to the device's stream-ordered pool.  Launches of a
 * captured graph that read the tree are not tracked: the caller waits for
 * them before freeing.  NULL is OK. */
int knn_tree_free(knn_tree* t);

/* knn_tree_errors -- waits for `stream`, then reads and clears the count of
 * queries that, since the previous call, named a tree id outside [0, trees)
 * in knn_query_batch (each was answered with padding rows).  bad_queries (may
 * be NULL) receives the count.  Returns KNN_EINVAL, with the count in the
 * message, when it is nonzero; KNN_OK otherwise. */
int knn_tree_errors(const knn_tree* t, void* stream, int64_t* bad_queries);

/* Sizes and shape of a tree. */
int knn_tree_info(const knn_tree* t, knn_tree_info_t* info);

/* Copy the tree to host arrays (synchronous); used to check its invariants. */
int knn_tree_export(const knn_tree* t, knn_tree_host* h);

/* Builds take their scratch and the trees' memory from a cache of device
 * blocks kept by the library (per device), which gives memory a build or a
 * freed tree handed back to later builds instead of mapping fresh memory;
 * at most 96 GiB of unused blocks are kept.  Query workspaces and serving
 * batches come from a stream-ordered pool the library creates per device,
 * which keeps up to 8 GiB of freed memory mapped for the next call instead of
 * returning it at every synchronisation (the device's default pool is left as
 * it is, and serves a first call made under graph capture).  This call waits
 * for the current device, frees every unused block and trims both pools. */
int knn_release_memory(void);

/* Message describing the last failure of the calling thread. */
const char* knn_last_error(void);

/* Fixed name of a return code ("KNN_OK", "KNN_EINVAL", ...; "unknown" for any
 * other value).  The string is static. */
const char* knn_strerror(int code);

/* Per-phase device times of the most recent build and query on this thread,
 * in milliseconds, taken with HIP events on the call's stream while profiling
 * is enabled: knn_set_profiling(1) records the phase boundaries; 2 also
 * records an event before and after every launch of the build's partition
 * kernel (slots 9-11), which leaves the device idle a few microseconds per
 * event; 0 turns profiling off.  Slots:
 *   build: 0 ingest, 1 level passes (sample, histogram, split, partition),
 *          2 subtree finish in LDS, 3 node compaction and boxes, 4 total
 *   query: 5 locate home leaves, 6 group queries by leaf, 7 traversal, 8 total
 *   build partition kernel: 9 summed duration of its launches (ms),
 *          10 number of launches, 11 points it moved (millions) */
#define KNN_PHASES 12
int knn_set_profiling(int32_t enable);
int knn_get_profile(float* ms_out /* [KNN_PHASES] */);

#ifdef __cplusplus
}
#endif
#endif /* KNN_H */
