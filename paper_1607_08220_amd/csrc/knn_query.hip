// Batched exact k-NN queries on gfx950 (Algorithm 1, Sections III-B/III-C of
// arXiv 1607.08220): the one-wavefront-per-query traversal, the home-leaf
// search and grouping of the queries, the merge of two candidate lists,
// and the host side that picks a traversal form and launches it.  The
// traversal kernels themselves are in knn_traverse.h.
#include "knn_traverse.h"

namespace knn {
namespace {
using WaveFn = void (*)(TravArgs);

// Home leaf of every query: descend with the near-child rule (x < split
// left).  Queries are grouped by key = (first packed position of the home
// leaf) >> shift: buckets are contiguous in packed order, so key order is the
// tree's spatial order.  Each lane descends kLocQ queries at once (blocks of
// kBlock * kLocQ consecutive queries, lane t taking t, t + kBlock, ...), so
// that kLocQ independent node loads are in flight per step (two per lane:
// 0.454 ms for 2^22 queries on the clustered 2^26-point tree, against 0.61
// with one, 0.466 with four and 0.52 with eight).
constexpr int kLocQ = 2;

// In 4 dimensions the default takes the explicit stack from k = 16 on, for
// buckets of 16 or more points: on 2^28 plasma-like points with 2^24 of them
// as queries it answers k = 16 in 58.2 / 57.4 / 62.8 ms (buckets of 16 / 32 /
// 64) against 63.8 / 61.5 / 66.1 for the stack-free walk, while the walk stays
// ahead for buckets of 8 (a deeper tree, a longer stack: 72.0 against 89.3
// ms), at k = 8 (36.6 against 40.2 ms) and in 3 dimensions (clustered, 2^26
// points, 2^22 queries: 4.2 against 5.5 ms at k = 8, 6.3 against 7.7 at 16).
constexpr int kStackMinK4 = 16;
constexpr int kStackMinLeaf4 = 16;

// Counting sort of the queries: scan blocks of kScanChunk bucket counts.
constexpr int kScanItems = 16;
constexpr int kScanChunk = kBlock * kScanItems;

// A query whose tree id is out of range descends tree 0 here (only its
// place in the grouped order depends on it); the traversal answers it with
// padding rows.
template <int D>
__global__ __launch_bounds__(kBlock) void k_locate(const NodeRec* __restrict__ nodes,
                                                   const float* __restrict__ queries,
                                                   const int32_t* __restrict__ qroot,
                                                   int32_t n_roots, int64_t m, int shift,
                                                   int32_t* __restrict__ home,
                                                   uint32_t* __restrict__ cnt)
{
    const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kLocQ) + threadIdx.x;
    float q[kLocQ][D];
    int cur[kLocQ];
    NodeRec r[kLocQ];
#pragma unroll
    for (int u = 0; u < kLocQ; ++u) {
        const int64_t i = min(i0 + (int64_t)u * kBlock, m - 1);  // clamped: extra lanes repeat
#pragma unroll
        for (int t = 0; t < D; ++t) q[u][t] = queries[i * D + t];
        const int rt = qroot ? qroot[i] : 0;
        cur[u] = (unsigned)rt < (unsigned)n_roots ? rt : 0;
    }
#pragma unroll
    for (int u = 0; u < kLocQ; ++u) r[u] = nodes[cur[u]];
    bool inner = false;
#pragma unroll
    for (int u = 0; u < kLocQ; ++u) inner = inner || r[u].dim >= 0;
    while (inner) {
        inner = false;
#pragma unroll
        for (int u = 0; u < kLocQ; ++u) {
            if (r[u].dim >= 0) {
                cur[u] = select_dim<D>(q[u], r[u].dim) < r[u].split ? r[u].a : r[u].a + 1;
                r[u] = nodes[cur[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < kLocQ; ++u) inner = inner || r[u].dim >= 0;
    }
#pragma unroll
    for (int u = 0; u < kLocQ; ++u) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        if (i < m) {
            home[i] = cur[u];
            atomicAdd(&cnt[r[u].a >> shift], 1u);
        }
    }
}

// Counting-sort scatter: query i takes the next slot of its home leaf's
// bucket, at the bucket's offset inside its scan block plus the block's base;
// slot p gets (i, home leaf) in one 8-byte store.
__global__ __launch_bounds__(kBlock) void k_group(const NodeRec* __restrict__ nodes,
                                                  const int32_t* __restrict__ home, int64_t m,
                                                  int shift, uint32_t* __restrict__ offs,
                                                  const uint32_t* __restrict__ bsum,
                                                  int2* __restrict__ slots)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int h = home[i];
    const int64_t key = nodes[h].a >> shift;
    const uint32_t p = atomicAdd(&offs[key], 1u) + bsum[key / kScanChunk];
    slots[p] = make_int2((int)i, h);
}

__global__ __launch_bounds__(kBlock) void k_zero(uint32_t* __restrict__ a, int64_t len)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < len) a[i] = 0u;
}

// Exclusive scan of the bucket counts: per-block scan of kScanChunk values in
// place and a scan of the block sums; k_group adds a bucket's block sum to
// the slot it takes.
__device__ uint32_t block_scan_excl(uint32_t v, uint32_t* wsum, uint32_t* total)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < w) base += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_local(uint32_t* __restrict__ a, int64_t len,
                                                       uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t wsum[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        v[r] = base + r < len ? a[base + r] : 0u;
        s += v[r];
    }
    uint32_t tot;
    uint32_t run = block_scan_excl(s, wsum, &tot);
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        if (base + r < len) a[base + r] = run;
        run += v[r];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t* __restrict__ bsum, int64_t nb)
{
    __shared__ uint32_t wsum[kBlock / 64];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_scan_excl(v, wsum, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}


using LocateFn = void (*)(const NodeRec*, const float*, const int32_t*, int32_t, int64_t, int,
                          int32_t*, uint32_t*);

StackFn stack_for(int d, int k, bool stats)
{
    return d <= 8 ? stack_for_low(d, k, stats) : stack_for_high(d, k, stats);
}

TraverseFn traverse_for(int d, int k, bool stats)
{
    return d <= 8 ? traverse_for_low(d, k, stats) : traverse_for_high(d, k, stats);
}

WaveFn wave_for(int d)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return k_traverse_wave<DD>;
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4)
        KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
        KNN_DIM_CASE(9) KNN_DIM_CASE(10) KNN_DIM_CASE(11) KNN_DIM_CASE(12)
        KNN_DIM_CASE(13) KNN_DIM_CASE(14) KNN_DIM_CASE(15) KNN_DIM_CASE(16)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
}

LocateFn locate_for(int d)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return k_locate<DD>;
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4)
        KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
        KNN_DIM_CASE(9) KNN_DIM_CASE(10) KNN_DIM_CASE(11) KNN_DIM_CASE(12)
        KNN_DIM_CASE(13) KNN_DIM_CASE(14) KNN_DIM_CASE(15) KNN_DIM_CASE(16)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
}

struct StreamBuf {
    void* p = nullptr;
    hipStream_t s = nullptr;
    ~StreamBuf()
    {
        if (p) (void)hipFreeAsync(p, s);
    }
};

// Workspace of knn_query_noalloc: a file-scope device array, so that those
// calls allocate nothing.  Each device holds its own copy from the first call
// there until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in): it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kNoAllocBytes = size_t(KNN_NOALLOC_WORKSPACE_BYTES);
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

}  // namespace

int noalloc_workspace(void** ptr, size_t* bytes)
{
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    KNN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(KNN_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {  // the current device is the one the call runs on
        void* p = nullptr;
        KNN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kNoAllocBytes;
    return KNN_OK;
}

namespace {

// One thread per query: a two-way merge of two ascending (D, idx) lists,
// skipping padding (idx < 0) and an entry equal to the one just written.
__global__ __launch_bounds__(kBlock) void k_merge(const int32_t* __restrict__ ia,
                                                  const float* __restrict__ da, int ka,
                                                  const int32_t* __restrict__ ib,
                                                  const float* __restrict__ db, int kb, int64_t m,
                                                  int k, int32_t* __restrict__ oi,
                                                  float* __restrict__ od)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= m) return;
    ia += q * ka;
    da += q * ka;
    ib += q * kb;
    db += q * kb;
    oi += q * k;
    od += q * k;
    int i = 0, j = 0, o = 0;
    int last_i = -1;
    float last_d = 0.0f;
    while (o < k) {
        const bool a_ok = i < ka && ia[i] >= 0;
        const bool b_ok = j < kb && ib[j] >= 0;
        if (!a_ok && !b_ok) break;
        bool take_a;
        if (!b_ok) take_a = true;
        else if (!a_ok) take_a = false;
        else take_a = da[i] < db[j] || (da[i] == db[j] && ia[i] <= ib[j]);
        const int id = take_a ? ia[i] : ib[j];
        const float dv = take_a ? da[i] : db[j];
        if (take_a) ++i;
        else ++j;
        if (o > 0 && id == last_i && dv == last_d) continue;  // the same entry in both lists
        oi[o] = id;
        od[o] = dv;
        last_i = id;
        last_d = dv;
        ++o;
    }
    for (; o < k; ++o) {
        oi[o] = -1;
        od[o] = INFINITY;
    }
}

}  // namespace

int merge_lists(const int32_t* ia, const float* da, int ka, const int32_t* ib, const float* db,
                int kb, int64_t m, int k, int32_t* oi, float* od, hipStream_t st)
{
    const unsigned grid = (unsigned)((m + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge, dim3(grid), dim3(kBlock), 0, st, ia, da, ka, ib, db, kb, m, k, oi, od);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

int note_tree_use(const knn_tree* t, hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    KNN_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return KNN_OK;  // a graph launch is the caller's to wait for
    std::lock_guard<std::mutex> g(t->use_mu);
    hipEvent_t ev = nullptr;
    for (auto& u : t->uses)
        if (u.first == st) ev = u.second;
    if (!ev) {
        KNN_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        t->uses.emplace_back(st, ev);
    }
    KNN_HIP(hipEventRecord(ev, st));
    return KNN_OK;
}

namespace {

// The traversal form query_tree takes for qs, and the sizes of its grouping.
struct FormChoice {
    bool use_team, use_wave, grouped;
    int trav;     // the asked form with an unusable team request dropped
    int team;     // lanes per query of the team form
    int shift;    // grouping key: packed position >> shift
    int64_t N;    // counting-sort buckets (0 without grouping)
    int64_t nsb;  // their scan blocks
    size_t bytes; // workspace
};

FormChoice choose_form(const knn_tree* t, const QuerySpec& qs)
{
    FormChoice f{};
    const int d = t->d;
    const int64_t m = qs.m;
    // one wavefront per query (the tree's depth bounds the lanes' stack):
    // asked for, or by default for batches too small to fill the device with
    // one lane per query; it runs in input order (grouping by home leaf costs
    // more than the coherence it buys a wavefront that walks one query)
    // a team of lanes per query: asked for, or by default for mid-size batches
    // of deep (high-dimensional) searches; k and the tree's depth must fit
    const bool high = d >= kStackMinDim;
    const bool team_default = qs.traversal == 0 && high && m > kWaveQueriesMaxHigh &&
                              m <= kTeamQueriesMax;
    f.team = qs.team ? qs.team : kTeamDefault;
    f.use_team = (qs.traversal == 4 || team_default) && qs.stats == nullptr &&
                 qs.k <= f.team && t->depth + 1 <= f.team;
    f.trav = qs.traversal == 4 && !f.use_team ? 0 : qs.traversal;
    const bool wave_ok = t->depth + 1 <= kWave && qs.stats == nullptr;
    const int64_t wave_max = high ? kWaveQueriesMaxHigh : kWaveQueriesMax;
    f.use_wave = !f.use_team && wave_ok && (f.trav == 3 || (f.trav == 0 && m <= wave_max));
    f.grouped = qs.order != 1 && !f.use_wave;
    // key range: packed positions >> shift, at most 2^22 buckets
    while ((t->n >> f.shift) > (int64_t(1) << 22)) ++f.shift;
    f.N = f.grouped ? (t->n >> f.shift) + 1 : 0;
    f.nsb = (f.N + kScanChunk - 1) / kScanChunk;
    const int64_t mg = f.grouped ? m : 0;
    // workspace: slots[m] (int2), cnt[N], block sums[nsb], home[m]
    f.bytes = sizeof(int2) * (size_t)mg + sizeof(uint32_t) * (size_t)(f.N + f.nsb) +
              sizeof(int32_t) * (size_t)mg;
    return f;
}

}  // namespace

size_t query_workspace_bytes(const knn_tree* t, const QuerySpec& qs)
{
    return choose_form(t, qs).bytes;
}

int query_tree(const knn_tree* t, const QuerySpec& qs, hipStream_t st)
{
    const int d = t->d;
    const int64_t m = qs.m;
    TraverseFn tf = traverse_for(d, qs.k, qs.stats != nullptr);
    LocateFn lf = locate_for(d);
    if (!tf || !lf) return fail(KNN_EINVAL, "unsupported dimension");
    prof_mark(st, 5);
    const unsigned grid = (unsigned)((m + kBlock - 1) / kBlock);
    const unsigned tgrid = (unsigned)((grid + kXcds - 1) / kXcds * kXcds);  // multiple of 8
    const FormChoice f = choose_form(t, qs);
    const bool use_team = f.use_team, use_wave = f.use_wave, grouped = f.grouped;
    const int trav = f.trav, team = f.team, shift = f.shift;
    const int64_t N = f.N, nsb = f.nsb, mg = grouped ? m : 0;
    const size_t bytes = f.bytes;
    StreamBuf ws;
    ws.s = st;
    void* base = nullptr;
    if (bytes && qs.ws) {
        if (bytes > qs.ws_bytes)
            return fail(KNN_EINVAL, "the query needs " + std::to_string(bytes) +
                                        " bytes of workspace, the static workspace holds " +
                                        std::to_string(qs.ws_bytes) +
                                        " (order 1 needs none)");
        base = qs.ws;
    } else if (bytes) {
        KNN_HIP(work_alloc(&ws.p, bytes, st));
        base = ws.p;
    }
    int2* slots = static_cast<int2*>(base);  // first: 8-byte aligned
    uint32_t* cnt = reinterpret_cast<uint32_t*>(slots + mg);
    uint32_t* bsum = cnt + N;
    int32_t* home = reinterpret_cast<int32_t*>(bsum + nsb);
    if (grouped) {
        // cleared by a kernel, not a memset node, so the call can be captured in a graph
        k_zero<<<(unsigned)((N + kBlock - 1) / kBlock), kBlock, 0, st>>>(cnt, N);
        const unsigned lgrid = (unsigned)((m + kBlock * kLocQ - 1) / (kBlock * kLocQ));
        hipLaunchKernelGGL(lf, dim3(lgrid), dim3(kBlock), 0, st, t->nodes, qs.queries, qs.qroot,
                           t->n_trees, m, shift, home, cnt);
        KNN_HIP(hipGetLastError());
    }
    prof_mark(st, 6);
    if (grouped) {
        k_scan_local<<<(unsigned)nsb, kBlock, 0, st>>>(cnt, N, bsum);
        k_scan_sums<<<1, kBlock, 0, st>>>(bsum, nsb);
        k_group<<<grid, kBlock, 0, st>>>(t->nodes, home, m, shift, cnt, bsum, slots);
        KNN_HIP(hipGetLastError());
    }
    prof_mark(st, 7);
    TravArgs A{};
    A.nodes = t->nodes;
    A.bbox = t->bbox;
    A.pts = t->pts;
    A.queries = qs.queries;
    A.slots = grouped ? slots : nullptr;
    A.start_home = grouped;
    A.root = qs.qroot;
    A.n_roots = t->n_trees;
    A.bad = t->bad;
    A.self_ids = qs.self_ids;
    A.r2s = qs.r2s;
    A.qk = qs.qk;
    A.qout = qs.qout;
    A.r2 = qs.r2;
    A.k = qs.k;
    A.batch = qs.batch;
    A.m = m;
    A.out_idx = qs.out_idx;
    A.out_d2 = qs.out_d2;
    A.stats = qs.stats;
    // the explicit stack needs (depth + 1) entries of 8 bytes per lane in LDS
    const size_t stk_bytes = sizeof(int2) * (size_t)(t->depth + 1) * kBlock;
    const bool use_stack = stk_bytes <= kMaxStackLds &&
                           (trav == 2 || (trav == 0 && (d >= kStackMinDim ||
                                                        (d == 4 && qs.k >= kStackMinK4 &&
                                                         t->leaf >= kStackMinLeaf4))));
    if (use_team) {  // grouped order (when asked) for locality; each team starts at its root
        TraverseFn ft = team_for(d, team);
        if (!ft) return fail(KNN_EINVAL, "unsupported dimension or team size");
        A.start_home = false;
        const int64_t per_block = (int64_t)kWavesPerBlock * (kWave / team);
        hipLaunchKernelGGL(ft, dim3((unsigned)((m + per_block - 1) / per_block)), dim3(kBlock), 0,
                           st, A);
    } else if (use_wave) {
        WaveFn wf = wave_for(d);
        const unsigned wgrid = (unsigned)((m + kWavesPerBlock - 1) / kWavesPerBlock);
        hipLaunchKernelGGL(wf, dim3(wgrid), dim3(kBlock), 0, st, A);
    } else if (use_stack) {
        StackFn sf = stack_for(d, qs.k, qs.stats != nullptr);
        if (stk_bytes > 64 * 1024)
            KNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(sf),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)stk_bytes));
        hipLaunchKernelGGL(sf, dim3(tgrid), dim3(kBlock), stk_bytes, st, A, t->depth + 1);
    } else {
        hipLaunchKernelGGL(tf, dim3(tgrid), dim3(kBlock), 0, st, A);
    }
    KNN_HIP(hipGetLastError());
    prof_mark(st, 8);
    // (a call on the static workspace creates no event: the caller waits)
    return qs.ws ? KNN_OK : note_tree_use(t, st);
}

}  // namespace knn
