// C-ABI entry points of libknn.so: argument checks, error reporting, tree
// lifetime, export and profiling.  The arithmetic lives in knn_build.hip,
// knn_query.hip and knn_classify.hip; the serving loop in knn_serve.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "knn_internal.h"

namespace knn {

namespace {
thread_local std::string g_err;
thread_local Profiler g_prof;

constexpr int64_t kMaxPoints = int64_t(1) << 30;  // node ids stay below 2^31

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return KNN_ENOMEM;
    return KNN_EDEVICE;
}

Profiler& profiler() { return g_prof; }

namespace {
std::mutex g_cache_mu;
std::multimap<std::pair<int, size_t>, void*> g_cache_free;     // (device, bytes) -> block
std::unordered_map<void*, std::pair<int, size_t>> g_cache_all;  // every block the cache made
size_t g_cache_free_bytes = 0;
constexpr size_t kCacheRound = size_t(2) << 20;
constexpr size_t kCacheKeepMax = size_t(96) << 30;  // free blocks kept beyond this are freed

// Free kept blocks of `dev` (all of them when dev < 0), largest first,
// until at most `keep` bytes stay.  The caller holds g_cache_mu.
hipError_t cache_shrink(int dev, size_t keep)
{
    hipError_t err = hipSuccess;
    for (auto it = g_cache_free.end(); it != g_cache_free.begin() && g_cache_free_bytes > keep;) {
        --it;
        if (dev >= 0 && it->first.first != dev) continue;
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (prev != it->first.first) (void)hipSetDevice(it->first.first);
        const hipError_t e = hipFree(it->second);
        if (prev != it->first.first) (void)hipSetDevice(prev);
        if (e != hipSuccess) err = e;
        g_cache_free_bytes -= it->first.second;
        g_cache_all.erase(it->second);
        it = g_cache_free.erase(it);
    }
    return err;
}
}  // namespace

hipError_t cache_alloc(void** out, size_t bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t want = (std::max<size_t>(bytes, 1) + kCacheRound - 1) / kCacheRound * kCacheRound;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_cache_free.lower_bound({dev, want});
        // a kept block of this device at most a quarter larger than asked for
        if (it != g_cache_free.end() && it->first.first == dev &&
            it->first.second <= want + want / 4 + kCacheRound) {
            *out = it->second;
            g_cache_free_bytes -= it->first.second;
            g_cache_free.erase(it);
            return hipSuccess;
        }
    }
    e = hipMalloc(out, want);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {  // hand kept blocks back, retry
        {
            std::lock_guard<std::mutex> g(g_cache_mu);
            (void)cache_shrink(dev, 0);
        }
        (void)hipGetLastError();
        e = hipMalloc(out, want);
    }
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_cache_all[*out] = {dev, want};
    return hipSuccess;
}

void cache_free(void* p)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto it = g_cache_all.find(p);
    if (it == g_cache_all.end()) return;  // not a cache block
    g_cache_free.emplace(it->second, p);
    g_cache_free_bytes += it->second.second;
    if (g_cache_free_bytes > kCacheKeepMax) (void)cache_shrink(-1, kCacheKeepMax);
}

// Bytes of freed memory the library's pool keeps mapped between calls.
constexpr uint64_t kPoolKeep = 8ull << 30;

// The library's stream-ordered pool of the current device: with `create`,
// made at the first call whose stream is not being captured; *out = NULL
// while none exists.
hipError_t work_pool(hipStream_t st, bool create, hipMemPool_t* out)
{
    static std::mutex mu;
    static std::vector<hipMemPool_t> pools;
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)pools.size() > dev && pools[dev]) {
        *out = pools[dev];
        return hipSuccess;
    }
    if (!create) return hipSuccess;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess || cs != hipStreamCaptureStatusNone) return e;
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    e = hipMemPoolCreate(&pool, &props);
    if (e != hipSuccess) return e;
    uint64_t keep = kPoolKeep;
    e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) return e;
    if ((int)pools.size() <= dev) pools.resize(dev + 1, nullptr);
    pools[dev] = pool;
    *out = pool;
    return hipSuccess;
}

hipError_t work_alloc(void** p, size_t bytes, hipStream_t st)
{
    hipMemPool_t pool = nullptr;
    hipError_t e = work_pool(st, true, &pool);
    if (e != hipSuccess) return e;
    // no pool yet during a first use under capture: the device's default pool
    return pool ? hipMallocFromPoolAsync(p, bytes, pool, st) : hipMallocAsync(p, bytes, st);
}

hipError_t cache_trim()
{
    std::lock_guard<std::mutex> g(g_cache_mu);
    return cache_shrink(-1, 0);
}

void prof_mark(hipStream_t s, int slot)
{
    if (!g_prof.on) return;
    if (!g_prof.ev[slot]) (void)hipEventCreate(&g_prof.ev[slot]);
    if (hipEventRecord(g_prof.ev[slot], s) == hipSuccess) g_prof.have[slot] = true;
}

void prof_part_begin()
{
    g_prof.part_used = 0;
    g_prof.part_points = 0.0;
}

void prof_part_mark(hipStream_t s)
{
    if (!g_prof.on || !g_prof.part) return;
    if (g_prof.part_used == (int)g_prof.part_ev.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return;
        g_prof.part_ev.push_back(e);
    }
    if (hipEventRecord(g_prof.part_ev[g_prof.part_used], s) == hipSuccess) ++g_prof.part_used;
}

void prof_part_points(double points) { g_prof.part_points = points; }

static int32_t pow2_floor(int32_t v)
{
    int32_t p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

// Largest per-wavefront subtree that fits the device's LDS per block.
static int32_t subtree_points_for(int32_t d, int32_t requested)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    size_t lds_max = 64 * 1024;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.sharedMemPerBlock > 0)
        lds_max = prop.sharedMemPerBlock;
    int32_t w = requested > 0 ? pow2_floor(std::min(requested, kSampleMax)) : default_subtree_points(d);
    w = std::min(w, finish_max_points(d));
    while (w > 64 && finish_lds_bytes_per_wave(d, finish_tile_points(d, w)) * 4 > lds_max) w >>= 1;
    return std::max(w, 64);
}

}  // namespace knn

using namespace knn;

extern "C" {

const char* knn_last_error(void) { return g_err.c_str(); }

const char* knn_strerror(int code)
{
    switch (code) {
    case KNN_OK: return "KNN_OK";
    case KNN_EINVAL: return "KNN_EINVAL";
    case KNN_ENOMEM: return "KNN_ENOMEM";
    case KNN_EDEVICE: return "KNN_EDEVICE";
    case KNN_EDEPTH: return "KNN_EDEPTH";
    case KNN_ENOTFINITE: return "KNN_ENOTFINITE";
    default: return "unknown";
    }
}

namespace {

// Build parameters with defaults filled in (max_depth stays 0 if unset).
struct BuildArgs {
    int32_t leaf, max_depth, W;
    int64_t sbn;
};

int build_args(int32_t dim, const knn_build_params* p, BuildArgs* a)
{
    if (dim < 1 || dim > KNN_MAX_DIM) return fail(KNN_EINVAL, "dim must be in [1, 16]");
    knn_build_params q = p ? *p : knn_build_params{0, 0, 0, 0};
    if (q.leaf_size < 0 || q.max_depth < 0 || q.subtree_points < 0 || q.split_block_nodes < -1)
        return fail(KNN_EINVAL, "negative build parameter");
    if (q.max_depth > 4096) return fail(KNN_EINVAL, "max_depth too large");
    a->leaf = q.leaf_size ? q.leaf_size : kDefaultLeaf;
    a->max_depth = q.max_depth;
    a->W = subtree_points_for(dim, q.subtree_points);
    a->sbn = q.split_block_nodes ? std::max(q.split_block_nodes, 0) : kDefaultSplitBlockNodes;
    return KNN_OK;
}

// offsets[0 .. trees]: 0, strictly increasing (every tree holds a point), at most 2^30.
int check_offsets(const int64_t* offsets, int32_t trees)
{
    if (!offsets) return fail(KNN_EINVAL, "offsets is NULL");
    if (trees < 1) return fail(KNN_EINVAL, "trees must be >= 1");
    if (offsets[0] != 0) return fail(KNN_EINVAL, "offsets[0] must be 0");
    for (int32_t t = 0; t < trees; ++t)
        if (offsets[t + 1] <= offsets[t]) return fail(KNN_EINVAL, "every tree needs >= 1 point");
    if (offsets[trees] > kMaxPoints) return fail(KNN_EINVAL, "more than 2^30 points in all");
    return KNN_OK;
}

int build_common(const float* points, int64_t n, int32_t dim, const int64_t* offsets,
                 int32_t trees, const knn_build_params* p, void* stream, knn_tree** out)
{
    if (!out) return fail(KNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!points) return fail(KNN_EINVAL, "points is NULL");
    if (n < 1 || n > kMaxPoints) return fail(KNN_EINVAL, "n must be in [1, 2^30]");
    BuildArgs a{};
    if (int rc = build_args(dim, p, &a)) return rc;
    return build_tree(points, n, dim, a.leaf, a.max_depth ? a.max_depth : kDefaultMaxDepth, a.W,
                      a.sbn, offsets, trees, static_cast<hipStream_t>(stream), out);
}

}  // namespace

int knn_build_ex(const float* points, int64_t n, int32_t dim, const knn_build_params* p,
                 void* stream, knn_tree** out)
{
    const int64_t offsets[2] = {0, n};
    return build_common(points, n, dim, offsets, 1, p, stream, out);
}

int knn_build_batch(const float* points, const int64_t* offsets, int32_t trees, int32_t dim,
                    const knn_build_params* p, void* stream, knn_tree** out)
{
    if (out) *out = nullptr;
    if (int rc = check_offsets(offsets, trees)) return rc;
    return build_common(points, offsets[trees], dim, offsets, trees, p, stream, out);
}

int knn_build_plan_create(int64_t n, int32_t dim, const int64_t* offsets, int32_t trees,
                          const knn_build_params* p, void* stream, knn_build_plan** out)
{
    if (!out) return fail(KNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxPoints) return fail(KNN_EINVAL, "n must be in [1, 2^30]");
    const int64_t one[2] = {0, n};
    if (!offsets) {
        if (trees != 1) return fail(KNN_EINVAL, "offsets is NULL with trees != 1");
        offsets = one;
    }
    if (int rc = check_offsets(offsets, trees)) return rc;
    if (offsets[trees] != n) return fail(KNN_EINVAL, "offsets[trees] must equal n");
    BuildArgs a{};
    if (int rc = build_args(dim, p, &a)) return rc;
    return plan_create(n, dim, offsets, trees, a.leaf, a.max_depth, a.W, a.sbn,
                       static_cast<hipStream_t>(stream), out);
}

int knn_build_plan_run(knn_build_plan* plan, const float* points, void* stream)
{
    if (!plan) return fail(KNN_EINVAL, "plan is NULL");
    if (!points) return fail(KNN_EINVAL, "points is NULL");
    DeviceGuard g(plan_device(plan));
    return plan_run(plan, points, static_cast<hipStream_t>(stream));
}

int knn_build_plan_finish(knn_build_plan* plan, void* stream, knn_tree** tree)
{
    if (tree) *tree = nullptr;
    if (!plan) return fail(KNN_EINVAL, "plan is NULL");
    DeviceGuard g(plan_device(plan));
    const int rc = plan_finish(plan, static_cast<hipStream_t>(stream));
    if (tree) *tree = plan_tree(plan);
    return rc;
}

knn_tree* knn_build_plan_tree(knn_build_plan* plan) { return plan ? plan_tree(plan) : nullptr; }

int knn_build_plan_destroy(knn_build_plan* plan)
{
    if (!plan) return KNN_OK;
    DeviceGuard g(plan_device(plan));
    return plan_destroy(plan);
}

int knn_build(const float* points, int64_t n, int32_t dim, int32_t leaf_size, void* stream,
              knn_tree** out)
{
    if (leaf_size < 0) return fail(KNN_EINVAL, "leaf_size must be >= 1");
    knn_build_params p{leaf_size, 0, 0, 0};
    return knn_build_ex(points, n, dim, &p, stream, out);
}

namespace {

int query_common(const knn_tree* t, const float* queries, int64_t m, int32_t k,
                 const int32_t* self_ids, float r2_max, const float* r2s, const int32_t* roots,
                 const knn_query_params* p, int32_t* out_idx, float* out_dist2, void* stream,
                 bool noalloc = false)
{
    if (!t) return fail(KNN_EINVAL, "tree is NULL");
    if (m < 0) return fail(KNN_EINVAL, "m must be >= 0");
    if (k < 1 || k > KNN_MAX_K) return fail(KNN_EINVAL, "k must be in [1, 64]");
    if (m > (int64_t(1) << 31) / KNN_MAX_K) return fail(KNN_EINVAL, "m too large");
    if (std::isnan(r2_max)) return fail(KNN_EINVAL, "r2_max is NaN");
    if (m == 0) return KNN_OK;
    if (!queries || !out_idx || !out_dist2) return fail(KNN_EINVAL, "NULL query or output pointer");
    const int32_t order = p ? p->order : 0;
    if (order != 0 && order != 1) return fail(KNN_EINVAL, "order must be 0 or 1");
    const int32_t batch = p && p->leaf_batch ? p->leaf_batch : kDefaultLeafBatch;
    if (batch < 1 || batch > 64) return fail(KNN_EINVAL, "leaf_batch must be in [0, 64]");
    const int32_t traversal = p ? p->traversal : 0;
    if (traversal < 0 || traversal > 4) return fail(KNN_EINVAL, "traversal must be 0 .. 4");
    const int32_t team = p ? p->team_lanes : 0;
    if (team != 0 && team != 8 && team != 16 && team != 32)
        return fail(KNN_EINVAL, "team_lanes must be 0, 8, 16 or 32");
    DeviceGuard g(t->device);
    QuerySpec qs;
    qs.queries = queries;
    qs.m = m;
    qs.k = k;
    qs.self_ids = self_ids;
    qs.r2 = r2_max;
    qs.r2s = r2s;
    qs.qroot = roots;
    qs.order = order;
    qs.batch = batch;
    qs.traversal = traversal;
    qs.team = team;
    qs.out_idx = out_idx;
    qs.out_d2 = out_dist2;
    qs.stats = p ? reinterpret_cast<unsigned long long*>(p->stats) : nullptr;
    if (noalloc) {  // the device's static workspace instead of an allocation
        const int rc = noalloc_workspace(&qs.ws, &qs.ws_bytes);
        if (rc != KNN_OK) return rc;
    }
    return query_tree(t, qs, static_cast<hipStream_t>(stream));
}

}  // namespace

int knn_query_ex(const knn_tree* t, const float* queries, int64_t m, int32_t k,
                 const int32_t* self_ids, float r2_max, const knn_query_params* p,
                 int32_t* out_idx, float* out_dist2, void* stream)
{
    if (t && t->n_trees != 1) return fail(KNN_EINVAL, "a forest is queried with knn_query_batch");
    return query_common(t, queries, m, k, self_ids, r2_max, nullptr, nullptr, p, out_idx,
                        out_dist2, stream);
}

int knn_query_noalloc(const knn_tree* t, const float* queries, int64_t m, int32_t k,
                      const int32_t* self_ids, float r2_max, const knn_query_params* p,
                      int32_t* out_idx, float* out_dist2, void* stream)
{
    if (t && t->n_trees != 1) return fail(KNN_EINVAL, "a forest is queried with knn_query_batch");
    return query_common(t, queries, m, k, self_ids, r2_max, nullptr, nullptr, p, out_idx,
                        out_dist2, stream, true);
}

int knn_query_batch(const knn_tree* t, const float* queries, const int32_t* tree_ids,
                    int64_t m, int32_t k, const int32_t* self_ids, float r2_max,
                    const knn_query_params* p, int32_t* out_idx, float* out_dist2, void* stream)
{
    if (m > 0 && !tree_ids) return fail(KNN_EINVAL, "tree_ids is NULL");
    return query_common(t, queries, m, k, self_ids, r2_max, nullptr, tree_ids, p, out_idx,
                        out_dist2, stream);
}

int knn_query_radius(const knn_tree* t, const float* queries, int64_t m, int32_t k,
                     const int32_t* self_ids, const float* r2, const knn_query_params* p,
                     int32_t* out_idx, float* out_dist2, void* stream)
{
    if (m > 0 && !r2) return fail(KNN_EINVAL, "r2 is NULL");
    if (t && t->n_trees != 1) return fail(KNN_EINVAL, "a forest is queried with knn_query_batch");
    return query_common(t, queries, m, k, self_ids, INFINITY, r2, nullptr, p, out_idx, out_dist2,
                        stream);
}

int knn_merge(const int32_t* idx_a, const float* dist2_a, int32_t ka, const int32_t* idx_b,
              const float* dist2_b, int32_t kb, int64_t m, int32_t k, int32_t* out_idx,
              float* out_dist2, void* stream)
{
    if (m < 0) return fail(KNN_EINVAL, "m must be >= 0");
    if (k < 1 || k > KNN_MAX_K || ka < 1 || ka > KNN_MAX_K || kb < 1 || kb > KNN_MAX_K)
        return fail(KNN_EINVAL, "ka, kb and k must be in [1, 64]");
    if (m == 0) return KNN_OK;
    if (!idx_a || !dist2_a || !idx_b || !dist2_b || !out_idx || !out_dist2)
        return fail(KNN_EINVAL, "NULL list pointer");
    return merge_lists(idx_a, dist2_a, ka, idx_b, dist2_b, kb, m, k, out_idx, out_dist2,
                       static_cast<hipStream_t>(stream));
}

int knn_query(const knn_tree* t, const float* queries, int64_t m, int32_t k, int32_t* out_idx,
              float* out_dist2, void* stream)
{
    return knn_query_ex(t, queries, m, k, nullptr, INFINITY, nullptr, out_idx, out_dist2, stream);
}

int knn_tree_free(knn_tree* t)
{
    if (!t) return KNN_OK;
    if (t->plan_owned) return fail(KNN_EINVAL, "the tree belongs to a build plan");
    DeviceGuard g(t->device);
    int rc = KNN_OK;
    {   // wait for the latest query on every stream that queried the tree; the
        // build synchronised its own stream before returning
        std::lock_guard<std::mutex> lk(t->use_mu);
        for (auto& u : t->uses) {
            hipError_t e = hipEventSynchronize(u.second);
            if (e != hipSuccess && rc == KNN_OK) rc = hip_fail(e, "hipEventSynchronize");
            (void)hipEventDestroy(u.second);
        }
        t->uses.clear();
    }
    // no work reads the tree's blocks any more: back to the cache for the
    // next build
    cache_free(t->pts);
    cache_free(t->nodes);
    cache_free(t->bbox);
    cache_free(t->bad);
    delete t;
    return rc;
}

int knn_tree_errors(const knn_tree* t, void* stream, int64_t* bad_queries)
{
    if (!t) return fail(KNN_EINVAL, "tree is NULL");
    DeviceGuard g(t->device);
    unsigned long long c = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    KNN_HIP(hipMemcpyAsync(&c, t->bad, sizeof(c), hipMemcpyDeviceToHost, st));
    KNN_HIP(hipMemsetAsync(t->bad, 0, sizeof(c), st));
    KNN_HIP(hipStreamSynchronize(st));
    if (bad_queries) *bad_queries = (int64_t)c;
    if (c) return fail(KNN_EINVAL, std::to_string(c) + " queries named a tree id outside [0, " +
                                       std::to_string(t->n_trees) + ") and got padding rows");
    return KNN_OK;
}

int knn_tree_info(const knn_tree* t, knn_tree_info_t* info)
{
    if (!t || !info) return fail(KNN_EINVAL, "NULL argument");
    info->n = t->n;
    info->dim = t->d;
    info->leaf_size = t->leaf;
    info->depth = t->depth;
    info->subtree_points = t->sub_pts;
    info->nodes = t->n_nodes;
    info->leaves = (t->n_nodes + t->n_trees) / 2;  // full binary trees
    info->device_bytes = t->bytes;
    info->trees = t->n_trees;
    info->pad_ = 0;
    return KNN_OK;
}

int knn_tree_export(const knn_tree* t, knn_tree_host* h)
{
    if (!t || !h) return fail(KNN_EINVAL, "NULL argument");
    DeviceGuard g(t->device);
    const int64_t N = t->n_nodes, n = t->n;
    const int d = t->d;
    std::vector<NodeRec> nodes(N);
    std::vector<float> bbox((size_t)N * 2 * d);
    std::vector<float> pts((size_t)n * (d + 1));
    KNN_HIP(hipDeviceSynchronize());
    KNN_HIP(hipMemcpy(nodes.data(), t->nodes, sizeof(NodeRec) * N, hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(bbox.data(), t->bbox, sizeof(float) * bbox.size(), hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(pts.data(), t->pts, sizeof(float) * pts.size(), hipMemcpyDeviceToHost));
    std::vector<int32_t> start(N), count(N);
    // children always carry larger ids than their parent
    for (int64_t v = N - 1; v >= 0; --v) {
        const NodeRec& r = nodes[v];
        if (r.dim < 0) {
            start[v] = r.a;
            count[v] = -r.dim;
        } else {
            if (r.a <= v || r.a + 1 >= N) return fail(KNN_EDEVICE, "corrupt node record");
            start[v] = start[r.a];
            count[v] = count[r.a] + count[r.a + 1];
        }
    }
    for (int64_t v = 0; v < N; ++v) {
        const NodeRec& r = nodes[v];
        if (h->dim) h->dim[v] = r.dim >= 0 ? r.dim : -1;
        if (h->split) h->split[v] = r.dim >= 0 ? r.split : 0.0f;
        if (h->left) h->left[v] = r.dim >= 0 ? r.a : -1;
        if (h->parent) h->parent[v] = r.parent;
        if (h->start) h->start[v] = start[v];
        if (h->count) h->count[v] = count[v];
        for (int j = 0; j < d; ++j) {
            if (h->lo) h->lo[v * d + j] = bbox[(size_t)v * 2 * d + j];
            if (h->hi) h->hi[v * d + j] = bbox[(size_t)v * 2 * d + d + j];
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        const float* row = &pts[(size_t)i * (d + 1)];
        if (h->perm) {
            int32_t id;
            std::memcpy(&id, row + d, sizeof(id));
            h->perm[i] = id;
        }
        if (h->packed)
            for (int j = 0; j < d; ++j) h->packed[i * d + j] = row[j];
    }
    return KNN_OK;
}

int knn_release_memory(void)
{
    int dev = 0;
    KNN_HIP(hipGetDevice(&dev));
    KNN_HIP(hipDeviceSynchronize());
    KNN_HIP(cache_trim());
    hipMemPool_t pool;
    KNN_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
    KNN_HIP(hipMemPoolTrimTo(pool, 0));
    KNN_HIP(work_pool(nullptr, false, &pool));
    if (pool) KNN_HIP(hipMemPoolTrimTo(pool, 0));
    return KNN_OK;
}

int knn_set_profiling(int32_t enable)
{
    g_prof.on = enable != 0;
    g_prof.part = enable >= 2;
    for (int i = 0; i < KNN_PHASES + 4; ++i) g_prof.have[i] = false;
    return KNN_OK;
}

int knn_get_profile(float* ms_out)
{
    if (!ms_out) return fail(KNN_EINVAL, "NULL argument");
    // (phase, first event, last event)
    static const int spans[9][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {0, 4},
                                    {5, 6}, {6, 7}, {7, 8}, {5, 8}};
    float part = 0.0f;
    const int pairs = g_prof.part_used / 2;
    for (int i = 0; i < pairs; ++i) {
        float ms = 0.0f;
        KNN_HIP(hipEventSynchronize(g_prof.part_ev[2 * i + 1]));
        KNN_HIP(hipEventElapsedTime(&ms, g_prof.part_ev[2 * i], g_prof.part_ev[2 * i + 1]));
        part += ms;
    }
    ms_out[9] = pairs ? part : -1.0f;
    ms_out[10] = (float)pairs;
    ms_out[11] = (float)(g_prof.part_points / 1e6);
    for (int p = 0; p < 9; ++p) {
        const int a = spans[p][0], b = spans[p][1];
        float ms = -1.0f;
        if (g_prof.have[a] && g_prof.have[b]) {
            KNN_HIP(hipEventSynchronize(g_prof.ev[b]));
            KNN_HIP(hipEventElapsedTime(&ms, g_prof.ev[a], g_prof.ev[b]));
        }
        ms_out[p] = ms;
    }
    return KNN_OK;
}

}  // extern "C"
