// Internal declarations shared by the build, query and API translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>
#include <string>
#include <utility>
#include <vector>

#include "knn.h"

namespace knn {

// Tree node, 16 bytes.  Inner node: a = left child id (the right child is
// a + 1), dim = split dimension (>= 0), split = split value.  Leaf: a = first
// packed position, dim = -(point count) (< 0), split unused.  parent = -1 at
// the root.
struct NodeRec {
    int32_t a;
    int32_t parent;
    float split;
    int32_t dim;
};
static_assert(sizeof(NodeRec) == 16, "NodeRec must stay 16 bytes");

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kSampleMax = 1024;   // sample points per node (Section III-A1)
constexpr int kDefaultLeaf = 32;   // bucket size the paper found best
constexpr int kDefaultMaxDepth = 64;
constexpr int64_t kDefaultSplitBlockNodes = 256;  // see knn_build_params.split_block_nodes
// lanes of 64 holding a bucket before a wavefront scans (knn_query_params.leaf_batch)
constexpr int kDefaultLeafBatch = 48;
// zero rows after the last bucket row: whole row batches may be loaded
constexpr int kRowPad = 8;

}  // namespace knn

// The tree owns every device buffer below.
struct knn_tree {
    int64_t n = 0;
    int32_t d = 0;
    int32_t leaf = 0;
    int32_t depth = 0;
    int32_t sub_pts = 0;
    int32_t n_trees = 1;             // a forest's tree t has root node t
    int64_t n_nodes = 0;
    int64_t n_leaves = 0;
    int32_t device = 0;
    float* pts = nullptr;            // [n][d+1]: packed coordinates, last word = index bits
    knn::NodeRec* nodes = nullptr;   // [n_nodes]
    float* bbox = nullptr;           // [n_nodes][2d]: lo[0..d), hi[0..d)
    // [1] count of queries that named a tree id outside [0, n_trees) since
    // knn_tree_errors last read it
    unsigned long long* bad = nullptr;
    int64_t bytes = 0;
    // Every stream that queried the tree, with an event recorded after its
    // latest query there: knn_tree_free waits for these and nothing else.
    mutable std::mutex use_mu;
    mutable std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
    // held by a build plan, whose runs rewrite it in place: freed with the plan
    bool plan_owned = false;
};

namespace knn {

// Thread-local error reporting.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define KNN_HIP(expr)                                              \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return ::knn::hip_fail(e_, #expr);   \
    } while (0)

// Device memory of builds and trees.  Blocks handed back here are kept per
// device and given out again to later requests of about the same size:
// mapping fresh device memory (tens of GiB for the largest builds) costs more
// than a build, and the stream-ordered pool returns its memory to the device
// at synchronisations.  A block is handed back only when no work on it
// remains.  cache_trim frees every kept block.
hipError_t cache_alloc(void** p, size_t bytes);
void cache_free(void* p);
hipError_t cache_trim();

// Device buffer owned by a scope.  With a stream it comes from the cache
// above and goes back there once that stream has finished with it; without
// one it is a plain allocation.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    bool cached = false;
    DevBuf() = default;
    explicit DevBuf(hipStream_t s) : stream(s), cached(true) {}
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    hipError_t alloc(size_t b) {
        reset();
        bytes = b;
        if (!b) return hipSuccess;
        return cached ? cache_alloc(&p, b) : hipMalloc(&p, b);
    }
    void reset() {
        if (p) {
            if (cached) {
                (void)hipStreamSynchronize(stream);  // nothing in flight may still use it
                cache_free(p);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
    }
    void* release() {
        void* q = p;
        p = nullptr;
        bytes = 0;
        return q;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Profiling: events recorded at phase boundaries on the call's stream.
struct Profiler {
    bool on = false;
    bool part = false;  // also time each launch of the build's partition kernel
    hipEvent_t ev[KNN_PHASES + 4] = {};
    bool have[KNN_PHASES + 4] = {};
    // events around each launch of the build's partition kernel
    std::vector<hipEvent_t> part_ev;
    int part_used = 0;
    double part_points = 0.0;
};
Profiler& profiler();
void prof_mark(hipStream_t s, int slot);
void prof_part_begin();                 // start of a build
void prof_part_mark(hipStream_t s);     // before / after one partition launch
void prof_part_points(double points);   // points moved by the build's partition launches

// Largest subtree (points) one wavefront finishes in LDS for dimension d.
int32_t default_subtree_points(int32_t d);
int32_t finish_max_points(int32_t d);
int32_t finish_tile_points(int32_t d, int32_t w);
size_t finish_lds_bytes_per_wave(int32_t d, int32_t w);

int build_tree(const float* points, int64_t n, int32_t d, int32_t leaf, int32_t max_depth,
               int32_t W, int64_t split_block_nodes, const int64_t* offsets, int32_t trees,
               hipStream_t stream, knn_tree** out);
// Build plans (knn_build_plan_*): max_depth 0 picks a bound from the largest
// tree's balanced depth.
int plan_create(int64_t n, int32_t d, const int64_t* offsets, int32_t trees, int32_t leaf,
                int32_t max_depth, int32_t W, int64_t split_block_nodes, hipStream_t stream,
                knn_build_plan** out);
int plan_run(knn_build_plan* plan, const float* points, hipStream_t stream);
int plan_finish(knn_build_plan* plan, hipStream_t stream);
int plan_destroy(knn_build_plan* plan);
knn_tree* plan_tree(knn_build_plan* plan);
int32_t plan_device(const knn_build_plan* plan);
// One batch of queries against a tree (or forest).  Per-query arrays are
// device pointers indexed by query; NULL selects the scalar.
struct QuerySpec {
    const float* queries = nullptr;  // [m][d]
    int64_t m = 0;
    int32_t k = 1;                   // k, or the largest per-query k
    const int32_t* self_ids = nullptr;
    float r2 = INFINITY;
    const float* r2s = nullptr;      // per-query squared radius
    const int32_t* qk = nullptr;     // per-query k
    const int64_t* qout = nullptr;   // per-query first output element
    const int32_t* qroot = nullptr;  // per-query root node (forests)
    int32_t order = 0;
    int32_t batch = 48;
    int32_t traversal = 0;           // 0 auto, 1 stack-free walk from the home leaf, 2 explicit
                                     // stack, 3 a wavefront per query, 4 a team per query
    int32_t team = 0;                // lanes per query of traversal 4 (0 = 32)
    int32_t* out_idx = nullptr;
    float* out_d2 = nullptr;
    unsigned long long* stats = nullptr;
    // caller-provided device workspace: when set the query allocates nothing
    // and fails with KNN_EINVAL before launching if it needs more than ws_bytes
    void* ws = nullptr;
    size_t ws_bytes = 0;
};

int query_tree(const knn_tree* t, const QuerySpec& qs, hipStream_t stream);
// Stream-ordered allocation of query and batch workspaces from the library's
// own pool on the current device, which keeps up to 8 GiB of freed memory
// mapped between calls (created at the first call outside a graph capture;
// the device's default pool serves a first call under capture).  Freed with
// hipFreeAsync.
hipError_t work_alloc(void** p, size_t bytes, hipStream_t stream);
hipError_t work_pool(hipStream_t stream, bool create, hipMemPool_t* out);
// Device workspace query_tree takes for qs (the grouping of queries by home
// leaf, when the traversal form it picks groups them); 0 otherwise.
size_t query_workspace_bytes(const knn_tree* t, const QuerySpec& qs);
// Record that `stream` has enqueued work reading the tree (skipped while the
// stream is being captured into a graph).
int note_tree_use(const knn_tree* t, hipStream_t stream);
// Device address and size of knn_query_noalloc's static workspace on the
// current device.
int noalloc_workspace(void** ptr, size_t* bytes);
int merge_lists(const int32_t* ia, const float* da, int ka, const int32_t* ib, const float* db,
                int kb, int64_t m, int k, int32_t* oi, float* od, hipStream_t stream);

}  // namespace knn
