// Serving loop: resident trees, continuous batching of query requests.
//
// Requests (a query batch of any size against one resident tree, with its
// own k) are queued by knn_server_submit from any host thread.  One worker
// thread per server admits them while the device works on earlier ones:
// pending requests for the same tree, whatever their k, are packed into one
// batch of up to kMaxBatchReqs requests and kMaxBatchQueries queries (each
// query carries its own k and output offset into the traversal, whose heap
// holds the batch's largest k), provided the batch's
// device memory fits in what the HBM budget leaves beside the batches in
// flight; each batch runs on one of the server's streams (gather the
// requests' queries, the traversal of Algorithm 1, scatter the results into
// each request's buffers) and retires when its event completes.  Batches in
// flight on different streams overlap on the device, and a request that
// arrives while they run joins the next batch as soon as memory and a stream
// are free.  Every query is answered by the same traversal as knn_query_ex,
// so a result is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "knn_traverse.h"

namespace {

constexpr int kMaxBatchReqs = 64;
constexpr int64_t kMaxBatchQueries = int64_t(1) << 18;
constexpr int kGroupMin = 2048;  // smaller batches skip the home-leaf grouping pass
constexpr int kBlockS = 256;

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// The requests of one batch, passed by value to the gather/scatter kernels.
struct ReqTable {
    int32_t n;
    int32_t d;
    int32_t k[kMaxBatchReqs];          // neighbours asked for by request r
    int64_t start[kMaxBatchReqs + 1];  // first query of request r in the batch; start[n] = total
    int64_t ostart[kMaxBatchReqs + 1]; // first output entry of request r; ostart[n] = total
    const float* q[kMaxBatchReqs];
    const int32_t* self[kMaxBatchReqs];
    int32_t* oi[kMaxBatchReqs];
    float* od[kMaxBatchReqs];
};

// Largest r with off[r] <= i (off ascending, off[0] = 0).
__device__ inline int req_of(const int64_t* off, int n, int64_t i)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Copy every request's queries (and self ids, -1 where none) into the
// batch's contiguous staging arrays, with each query's k and the first entry
// of its row in the batch's packed output.
__global__ __launch_bounds__(kBlockS) void k_gather(ReqTable T, float* __restrict__ q,
                                                    int32_t* __restrict__ self,
                                                    int32_t* __restrict__ qk,
                                                    int64_t* __restrict__ qout)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= T.start[T.n]) return;
    const int r = req_of(T.start, T.n, i);
    const int64_t j = i - T.start[r];
    for (int t = 0; t < T.d; ++t) q[i * T.d + t] = T.q[r][j * T.d + t];
    self[i] = T.self[r] ? T.self[r][j] : -1;
    qk[i] = T.k[r];
    qout[i] = T.ostart[r] + j * T.k[r];
}

// Copy the batch's packed results into each request's own output buffers.
__global__ __launch_bounds__(kBlockS) void k_scatter_results(ReqTable T,
                                                             const int32_t* __restrict__ oi,
                                                             const float* __restrict__ od)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= T.ostart[T.n]) return;
    const int r = req_of(T.ostart, T.n, e);
    const int64_t o = e - T.ostart[r];
    T.oi[r][o] = oi[e];
    T.od[r][o] = od[e];
}

// ---------------------------------------------------------------------------
// Slot kernel: one persistent launch per tree answers small requests as they
// arrive.  The host posts a request (its query, self-id and output pointers,
// m and k) into a ring in coherent pinned host memory and bumps `posted`.
// Wavefront 0 of the launch (the dispatcher) takes posted requests over into
// device memory while the ring has room, and reports each request whose
// queries are all answered by a system-scope store of p + 1 into done[p].
// Every other wavefront (a worker) claims the next query of the admitted
// request with the fewest queries left to hand out (shortest first, so a
// small request that arrives behind a large one is answered within the
// time of one query), answers it with the one-wavefront-per-query traversal
// and counts it.  A launch stops admitting after a lifetime and ends when
// nothing is in flight, or after an idle time; the host relaunches it when
// requests are waiting.  The bounded lifetime keeps a launch from holding
// its hardware queue, which other streams may share, for long.
constexpr int kRing = 256;                  // requests in flight per slot kernel
constexpr int64_t kSlotMaxQueries = 16384;  // the largest request a slot kernel takes
constexpr int kSlotIdleUs = 2000;           // a launch with nothing to do ends after this
constexpr int kSlotWgPerCu = 1;             // workgroups of four wavefronts per compute unit
constexpr int kSlotLifeMs = 20;             // and stops admitting after this
constexpr int kSlotWords = 5;               // q, self, out idx, out dist, m | k << 32
constexpr int kSlotWatchdogMs = 5000;       // a launch fails what is in flight and ends
constexpr uint64_t kSlotFailed = uint64_t(1) << 63;  // done-word flag: the request was not answered
constexpr int kPersistBlock = 256;

struct PHost {                  // coherent pinned host memory
    uint64_t posted;            // host: requests posted; request p sits in ring[p % kRing]
    uint64_t consumed;          // device: requests taken over by a launch
    uint64_t stop;              // host: stop admitting
    uint64_t pad;
    uint64_t ring[kRing][kSlotWords];
    uint64_t tag[kRing];        // host: p + 1, written after request p's words
    uint64_t done[kRing];       // device: p + 1 once request p is answered (| kSlotFailed)
};

struct PDev {                   // device memory of one slot kernel
    uint64_t head;              // oldest request not yet reported
    uint64_t tail;              // requests handed to the workers
    uint64_t exit;              // the launch ends
    uint64_t pad;
    int32_t claim[kRing];       // next query to hand out
    int32_t finished[kRing];    // queries answered
    int32_t reported[kRing];
    uint64_t slot[kRing][kSlotWords];
};

// Shared words are read with relaxed scoped atomic loads: these bypass the
// compute unit's caches without invalidating the L2 that holds the tree.
__device__ inline uint64_t ld_sys(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline uint64_t ld_dev(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int32_t ld_dev(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline void st_dev(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void slot_dispatch(PHost* __restrict__ H, PDev* __restrict__ V, uint64_t idle_ticks,
                              uint64_t life_ticks, uint64_t watchdog_ticks)
{
    const int lane = threadIdx.x & (knn::kWave - 1);
    uint64_t head = ld_dev(&V->head), tail = ld_dev(&V->tail);
    const uint64_t t0 = wall_clock64();
    uint64_t busy_at = t0;
    bool admitting = true;
    while (true) {
        const uint64_t now = wall_clock64();
        if (admitting && (now - t0 > life_ticks || ld_sys(&H->stop))) admitting = false;
        if (now - t0 > watchdog_ticks) {  // never expected: fail what is in flight and end
            for (uint64_t p0 = head; p0 < tail; p0 += knn::kWave) {
                const uint64_t p = p0 + lane;
                if (p < tail && !ld_dev(&V->reported[p % kRing]))
                    __hip_atomic_store(&H->done[p % kRing], (p + 1) | kSlotFailed, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
            }
            if (lane == 0) st_dev(&V->exit, uint64_t(1));
            return;
        }
        if (admitting) {
            const uint64_t posted = ld_sys(&H->posted);
            uint64_t lim = posted < head + kRing ? posted : head + kRing;
            // take a request over only once its tag shows all its words written
            for (uint64_t p = tail; p < lim; ++p)
                if (ld_sys(&H->tag[p % kRing]) != p + 1) {
                    lim = p;
                    break;
                }
            if (tail < lim) {
                for (uint64_t p = tail; p < lim; ++p) {
                    const int sl = (int)(p % kRing);
                    if (lane < kSlotWords) st_dev(&V->slot[sl][lane], ld_sys(&H->ring[sl][lane]));
                }
                // the descriptors reach memory before their counters are reset
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                for (uint64_t p = tail; p < lim; ++p) {
                    const int sl = (int)(p % kRing);
                    if (lane == 0) {
                        st_dev(&V->claim[sl], 0);
                        st_dev(&V->finished[sl], 0);
                        st_dev(&V->reported[sl], 0);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                tail = lim;
                if (lane == 0) {
                    st_dev(&V->tail, tail);
                    __hip_atomic_store(&H->consumed, tail, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
        }
        // report the requests whose queries are all answered (the workers'
        // result rows were written back before their counts)
        for (uint64_t p0 = head; p0 < tail; p0 += knn::kWave) {
            const uint64_t p = p0 + lane;
            if (p < tail) {
                const int sl = (int)(p % kRing);
                const int m = (int)(uint32_t)ld_dev(&V->slot[sl][4]);
                if (!ld_dev(&V->reported[sl]) && ld_dev(&V->finished[sl]) == m) {
                    st_dev(&V->reported[sl], 1);
                    __hip_atomic_store(&H->done[sl], p + 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
        }
        while (head < tail && ld_dev(&V->reported[head % kRing])) ++head;
        if (lane == 0) st_dev(&V->head, head);
        if (head < tail) busy_at = now;
        if (head == tail && (!admitting || now - busy_at > idle_ticks)) {
            if (lane == 0) st_dev(&V->exit, uint64_t(1));  // requests still posted wait for the next launch
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

template <int D>
__device__ void slot_work(const knn::NodeRec* __restrict__ nodes, const float* __restrict__ bbox,
                          const float* __restrict__ pts, PDev* __restrict__ V)
{
    const int lane = threadIdx.x & (knn::kWave - 1);
    int nap = 1;  // idle polls back off, up to about 4 us apart
    while (true) {
        const uint64_t head = ld_dev(&V->head);
        const uint64_t tail = ld_dev(&V->tail);
        // the admitted request with the fewest queries left to hand out
        uint64_t best = ~0ull;  // (left << 32) | slot
        for (uint64_t p0 = head; p0 < tail; p0 += knn::kWave) {
            const uint64_t p = p0 + lane;
            uint64_t key = ~0ull;
            if (p < tail) {
                const int sl = (int)(p % kRing);
                const int m = (int)(uint32_t)ld_dev(&V->slot[sl][4]);
                const int c = ld_dev(&V->claim[sl]);
                if (c < m) key = ((uint64_t)(uint32_t)(m - c) << 32) | (uint32_t)sl;
            }
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)key, o);
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(key >> 32), o);
                const uint64_t y = ((uint64_t)hi << 32) | lo;
                key = y < key ? y : key;
            }
            best = key < best ? key : best;
        }
        if (best != ~0ull) {
            const int sl = __builtin_amdgcn_readfirstlane((int)(uint32_t)best);
            int qi = 0;
            if (lane == 0)
                qi = __hip_atomic_fetch_add(&V->claim[sl], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            qi = __builtin_amdgcn_readfirstlane(qi);
            const uint64_t mk = ld_dev(&V->slot[sl][4]);
            const int m = (int)(uint32_t)mk, k = (int)(mk >> 32);
            if (qi < m) {  // else the request's last queries went to other workers
                const float* qp = reinterpret_cast<const float*>(ld_dev(&V->slot[sl][0]));
                const int32_t* sp = reinterpret_cast<const int32_t*>(ld_dev(&V->slot[sl][1]));
                int32_t* oi = reinterpret_cast<int32_t*>(ld_dev(&V->slot[sl][2]));
                float* od = reinterpret_cast<float*>(ld_dev(&V->slot[sl][3]));
                if (qp && oi && od && k >= 1 && k <= knn::kWave) {  // (always: checked on submit)
                    // the caller wrote these while the launch ran: read past stale cached lines
                    float q[D];
#pragma unroll
                    for (int t = 0; t < D; ++t)
                        q[t] = __hip_atomic_load(qp + (int64_t)qi * D + t, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                    const int32_t self = sp ? __hip_atomic_load(sp + qi, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT)
                                            : -1;
                    knn::wave_answer<D>(nodes, bbox, pts, q, self, k, INFINITY, 0,
                                        oi + (int64_t)qi * k, od + (int64_t)qi * k);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // rows written back, then counted
                if (lane == 0)
                    __hip_atomic_fetch_add(&V->finished[sl], 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            nap = 1;
            continue;
        }
        if (ld_dev(&V->exit)) return;
        for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(127);
        nap = nap < 4 ? 2 * nap : 4;
    }
}

template <int D>
__global__ __launch_bounds__(kPersistBlock) void k_slots(const knn::NodeRec* nodes,
                                                         const float* bbox, const float* pts,
                                                         PHost* H, PDev* V, uint64_t idle_ticks,
                                                         uint64_t life_ticks, uint64_t watchdog_ticks)
{
    if (blockIdx.x == 0 && threadIdx.x < knn::kWave)
        slot_dispatch(H, V, idle_ticks, life_ticks, watchdog_ticks);
    else
        slot_work<D>(nodes, bbox, pts, V);
}

// Start of a launch: the window starts at the first request not yet taken.
__global__ void k_slots_init(PDev* V, uint64_t start)
{
    if (threadIdx.x == 0) {
        V->head = start;
        V->tail = start;
        V->exit = 0;
    }
}

using SlotFn = void (*)(const knn::NodeRec*, const float*, const float*, PHost*, PDev*, uint64_t,
                        uint64_t, uint64_t);

SlotFn slots_for(int d)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return k_slots<DD>;
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4)
        KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
        KNN_DIM_CASE(9) KNN_DIM_CASE(10) KNN_DIM_CASE(11) KNN_DIM_CASE(12)
        KNN_DIM_CASE(13) KNN_DIM_CASE(14) KNN_DIM_CASE(15) KNN_DIM_CASE(16)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
}

struct Request {
    int64_t ticket = 0;
    int32_t tree = 0;
    const float* q = nullptr;
    int64_t m = 0;
    int32_t k = 1;
    const int32_t* self = nullptr;
    int32_t* oi = nullptr;
    float* od = nullptr;
    double t_submit = 0.0, t_done = 0.0;
    int status = 1;  // 1 pending, 0 done, < 0 error code
};

struct Batch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* mem = nullptr;
    size_t bytes = 0;
    int32_t kmax = 1;
    int64_t queries = 0;
    int64_t outputs = 0;  // sum over requests of m * k
    std::vector<Request*> reqs;
    int status = KNN_OK;
};

}  // namespace

namespace {

// Host side of one tree's slot kernel.
struct SlotKernel {
    PHost* host = nullptr;   // coherent pinned host memory
    PDev* dev = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ended = nullptr;  // recorded after each launch
    bool launched = false;
    uint64_t posted = 0;
    std::vector<std::pair<uint64_t, Request*>> inflight;  // posted, not yet reported
};

}  // namespace

struct knn_server {
    std::vector<const knn_tree*> trees;
    int device = 0;
    int64_t budget = 0;
    // slot kernels (one per tree) for requests of at most slot_max queries
    int64_t slot_max = 0;  // 0: none
    std::vector<SlotKernel> slotk;
    int slot_blocks = 0;
    uint64_t idle_ticks = 0, life_ticks = 0, watchdog_ticks = 0;
    int64_t n_slot_requests = 0, n_slot_launches = 0;
    std::vector<hipStream_t> streams;
    std::vector<bool> busy;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::unordered_map<int64_t, Request*> reqs;
    int64_t next_ticket = 1;
    bool stop = false;
    std::vector<Batch> inflight;
    int64_t inflight_bytes = 0;
    // counters (knn_server_stats)
    int64_t n_batches = 0, n_queries = 0, n_requests = 0;
    int64_t peak_bytes = 0;
    int64_t max_reqs_per_batch = 0, peak_inflight = 0, max_k_kinds = 0;
    int64_t joined_running = 0;  // requests launched while an earlier batch was on the device
};

namespace {

// The query of a batch of `total` queries whose largest k is kmax (its
// device pointers are filled in at launch).
knn::QuerySpec batch_query(int64_t total, int32_t kmax)
{
    knn::QuerySpec qs;
    qs.m = total;
    qs.k = kmax;
    qs.order = total >= kGroupMin ? 0 : 1;
    qs.batch = knn::kDefaultLeafBatch;
    return qs;
}

// Device bytes a batch needs: staging for its queries, self ids, per-query
// k and output offsets, and results, plus the workspace of the query path
// (its grouping, when the traversal form it picks groups).
size_t batch_bytes(const knn_tree* t, int64_t total, int64_t outputs, int32_t kmax)
{
    return (size_t)total * (sizeof(float) * t->d + sizeof(int32_t) * 2 + sizeof(int64_t)) +
           (size_t)outputs * 8 + knn::query_workspace_bytes(t, batch_query(total, kmax));
}

int launch_batch(knn_server* s, Batch& b)
{
    const knn_tree* t = s->trees[b.reqs[0]->tree];
    const int d = t->d;
    ReqTable T{};
    T.n = (int32_t)b.reqs.size();
    T.d = d;
    int64_t total = 0, outs = 0;
    for (int r = 0; r < T.n; ++r) {
        const Request* q = b.reqs[r];
        T.start[r] = total;
        T.ostart[r] = outs;
        T.k[r] = q->k;
        T.q[r] = q->q;
        T.self[r] = q->self;
        T.oi[r] = q->oi;
        T.od[r] = q->od;
        total += q->m;
        outs += q->m * q->k;
    }
    T.start[T.n] = total;
    T.ostart[T.n] = outs;
    // staging: qout [total] int64, q [total][d], self [total], qk [total],
    // oi [outs], od [outs] (8-byte array first)
    const size_t b_qout = sizeof(int64_t) * total, b_q = sizeof(float) * total * d;
    const size_t b_i = sizeof(int32_t) * total, b_o = sizeof(int32_t) * outs;
    KNN_HIP(knn::work_alloc(&b.mem, b_qout + b_q + 2 * b_i + 2 * b_o, b.stream));
    char* base = static_cast<char*>(b.mem);
    int64_t* qout = reinterpret_cast<int64_t*>(base);
    float* q = reinterpret_cast<float*>(base + b_qout);
    int32_t* self = reinterpret_cast<int32_t*>(base + b_qout + b_q);
    int32_t* qk = reinterpret_cast<int32_t*>(base + b_qout + b_q + b_i);
    int32_t* oi = reinterpret_cast<int32_t*>(base + b_qout + b_q + 2 * b_i);
    float* od = reinterpret_cast<float*>(base + b_qout + b_q + 2 * b_i + b_o);
    const unsigned g1 = (unsigned)((total + kBlockS - 1) / kBlockS);
    k_gather<<<g1, kBlockS, 0, b.stream>>>(T, q, self, qk, qout);
    KNN_HIP(hipGetLastError());
    knn::QuerySpec qs = batch_query(total, b.kmax);
    qs.queries = q;
    qs.qk = qk;
    qs.qout = qout;
    qs.self_ids = self;
    qs.out_idx = oi;
    qs.out_d2 = od;
    const int rc = knn::query_tree(t, qs, b.stream);
    if (rc != KNN_OK) return rc;
    const unsigned g2 = (unsigned)((outs + kBlockS - 1) / kBlockS);
    k_scatter_results<<<g2, kBlockS, 0, b.stream>>>(T, oi, od);
    KNN_HIP(hipGetLastError());
    KNN_HIP(hipFreeAsync(b.mem, b.stream));
    b.mem = nullptr;
    KNN_HIP(hipEventRecord(b.done, b.stream));
    return KNN_OK;
}

bool slot_running(SlotKernel& k)
{
    return k.launched && hipEventQuery(k.ended) == hipErrorNotReady;
}

int slot_launch(knn_server* s, int tree)
{
    SlotKernel& k = s->slotk[tree];
    const knn_tree* t = s->trees[tree];
    const SlotFn f = slots_for(t->d);
    if (!f) return knn::fail(KNN_EINVAL, "unsupported dimension");
    // the requests taken over by earlier launches are all answered
    const uint64_t start = __atomic_load_n(&k.host->consumed, __ATOMIC_ACQUIRE);
    k_slots_init<<<1, knn::kWave, 0, k.stream>>>(k.dev, start);
    hipLaunchKernelGGL(f, dim3(s->slot_blocks), dim3(kPersistBlock), 0, k.stream, t->nodes, t->bbox,
                       t->pts, k.host, k.dev, s->idle_ticks, s->life_ticks, s->watchdog_ticks);
    KNN_HIP(hipGetLastError());
    KNN_HIP(hipEventRecord(k.ended, k.stream));
    k.launched = true;
    ++s->n_slot_launches;
    return KNN_OK;
}

// Post a request into its tree's ring; false when the ring has no room (the
// request kRing posts earlier is still in flight).
bool slot_post(knn_server* s, Request* r)
{
    SlotKernel& k = s->slotk[r->tree];
    uint64_t oldest = k.posted;
    for (const auto& e : k.inflight) oldest = std::min(oldest, e.first);
    if (k.posted - oldest >= (uint64_t)kRing) return false;
    const uint64_t p = k.posted;
    uint64_t* w = k.host->ring[p % kRing];
    w[0] = reinterpret_cast<uint64_t>(r->q);
    w[1] = reinterpret_cast<uint64_t>(r->self);
    w[2] = reinterpret_cast<uint64_t>(r->oi);
    w[3] = reinterpret_cast<uint64_t>(r->od);
    w[4] = (uint64_t)(uint32_t)r->m | ((uint64_t)(uint32_t)r->k << 32);
    __atomic_store_n(&k.host->tag[p % kRing], p + 1, __ATOMIC_RELEASE);
    __atomic_store_n(&k.host->posted, p + 1, __ATOMIC_RELEASE);
    k.posted = p + 1;
    k.inflight.emplace_back(p, r);
    return true;
}

// Retire the slot requests the kernels have answered; relaunch a kernel that
// ended while requests of its tree were still waiting.
bool slot_poll(knn_server* s)
{
    bool retired = false;
    for (size_t tr = 0; tr < s->slotk.size(); ++tr) {
        SlotKernel& k = s->slotk[tr];
        if (k.inflight.empty()) continue;
        const bool running = slot_running(k);  // before the flags: an ended launch wrote them all
        const double t = now_ms();
        for (size_t i = 0; i < k.inflight.size();) {
            const uint64_t p = k.inflight[i].first;
            const uint64_t dn = __atomic_load_n(&k.host->done[p % kRing], __ATOMIC_ACQUIRE);
            if ((dn & ~kSlotFailed) == p + 1) {
                Request* r = k.inflight[i].second;
                r->t_done = t;
                r->status = dn & kSlotFailed ? KNN_EDEVICE : KNN_OK;
                k.inflight[i] = k.inflight.back();
                k.inflight.pop_back();
                retired = true;
            } else {
                ++i;
            }
        }
        if (!k.inflight.empty() && !running) {
            const int rc = slot_launch(s, (int)tr);
            if (rc != KNN_OK) {  // the requests fail rather than wait forever
                for (auto& e : k.inflight) {
                    e.second->t_done = t;
                    e.second->status = rc;
                }
                k.inflight.clear();
                retired = true;
            }
        }
    }
    return retired;
}

bool slots_busy(knn_server* s)
{
    for (auto& k : s->slotk)
        if (!k.inflight.empty()) return true;
    return false;
}

void worker_loop(knn_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        // small requests go to their tree's slot kernel, in arrival order
        bool posted = false;
        if (s->slot_max > 0)
            for (auto it = s->pending.begin(); it != s->pending.end();) {
                Request* r = *it;
                if (r->m <= s->slot_max && slot_post(s, r)) {
                    if (slot_running(s->slotk[r->tree])) ++s->joined_running;
                    ++s->n_slot_requests;
                    s->n_queries += r->m;
                    it = s->pending.erase(it);
                    posted = true;
                } else {
                    ++it;
                }
            }
        bool retired = slot_poll(s);  // also launches a kernel for what was just posted
        (void)posted;
        // retire the batches whose work has completed
        for (size_t i = 0; i < s->inflight.size();) {
            Batch& b = s->inflight[i];
            const hipError_t e = b.status == KNN_OK ? hipEventQuery(b.done) : hipSuccess;
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            const double t = now_ms();
            const int st = b.status != KNN_OK ? b.status : (e == hipSuccess ? KNN_OK : KNN_EDEVICE);
            for (Request* r : b.reqs) {
                r->t_done = t;
                r->status = st;
            }
            s->inflight_bytes -= (int64_t)b.bytes;
            for (size_t j = 0; j < s->streams.size(); ++j)
                if (s->streams[j] == b.stream) s->busy[j] = false;
            (void)hipEventDestroy(b.done);
            s->inflight.erase(s->inflight.begin() + (std::ptrdiff_t)i);
            retired = true;
        }
        if (retired) s->cv_done.notify_all();
        // admit pending requests into new batches while a stream and memory are free
        // (with slot kernels, only the requests too large for them)
        while (!s->pending.empty()) {
            if (s->slot_max > 0 && s->pending.front()->m <= s->slot_max) break;  // waits for ring room
            int sidx = -1;
            for (size_t j = 0; j < s->streams.size(); ++j)
                if (!s->busy[j]) {
                    sidx = (int)j;
                    break;
                }
            if (sidx < 0) break;
            Request* head = s->pending.front();
            const knn_tree* t = s->trees[head->tree];
            Batch b;
            int64_t total = 0;
            uint64_t kinds = 0;  // bit k-1: some request asks for k neighbours
            for (auto it = s->pending.begin(); it != s->pending.end() && (int)b.reqs.size() < kMaxBatchReqs;) {
                Request* r = *it;
                if (r->tree == head->tree && (s->slot_max <= 0 || r->m > s->slot_max) &&
                    (b.reqs.empty() || total + r->m <= kMaxBatchQueries)) {
                    b.reqs.push_back(r);
                    total += r->m;
                    b.outputs += r->m * r->k;
                    b.kmax = std::max(b.kmax, r->k);
                    kinds |= uint64_t(1) << (r->k - 1);
                    it = s->pending.erase(it);
                } else {
                    ++it;
                }
            }
            b.queries = total;
            b.bytes = batch_bytes(t, total, b.outputs, b.kmax);
            if (!s->inflight.empty() && s->inflight_bytes + (int64_t)b.bytes > s->budget) {
                // not enough memory beside the batches in flight: wait for one to retire
                for (auto it = b.reqs.rbegin(); it != b.reqs.rend(); ++it) s->pending.push_front(*it);
                break;
            }
            b.stream = s->streams[sidx];
            s->busy[sidx] = true;
            (void)hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
            b.status = launch_batch(s, b);
            if (b.status != KNN_OK && b.mem) (void)hipFreeAsync(b.mem, b.stream);
            s->inflight_bytes += (int64_t)b.bytes;
            s->peak_bytes = std::max(s->peak_bytes, s->inflight_bytes);
            ++s->n_batches;
            s->n_queries += total;
            s->max_reqs_per_batch = std::max<int64_t>(s->max_reqs_per_batch, (int64_t)b.reqs.size());
            s->max_k_kinds = std::max<int64_t>(s->max_k_kinds, __builtin_popcountll(kinds));
            if (!s->inflight.empty()) s->joined_running += (int64_t)b.reqs.size();
            s->inflight.push_back(std::move(b));
            s->peak_inflight = std::max<int64_t>(s->peak_inflight, (int64_t)s->inflight.size());
        }
        if (s->stop && s->pending.empty() && s->inflight.empty() && !slots_busy(s)) break;
        if (s->inflight.empty() && !slots_busy(s) && s->pending.empty()) {
            s->cv_work.wait(lk, [s] { return s->stop || !s->pending.empty(); });
        } else {
            // poll the work in flight; new requests wake the loop as well
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

extern "C" {

int knn_server_create_ex(const knn_tree* const* trees, int32_t ntrees, const knn_server_params* p,
                         knn_server** out)
{
    if (!out) return knn::fail(KNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!trees || ntrees < 1) return knn::fail(KNN_EINVAL, "no trees");
    const knn_server_params q = p ? *p : knn_server_params{0, 0, 0, 0, 0};
    if (q.hbm_budget_bytes < 0 || q.streams < 0 || q.streams > 64 || q.slot_max_queries < 0 ||
        q.slot_workgroups_per_cu < 0 || q.slot_workgroups_per_cu > 8 || q.slot_idle_us < 0)
        return knn::fail(KNN_EINVAL, "budget must be >= 0, streams in [0, 64], slot_max_queries >= 0, "
                                     "slot_workgroups_per_cu in [0, 8], slot_idle_us >= 0");
    for (int32_t i = 0; i < ntrees; ++i) {
        if (!trees[i]) return knn::fail(KNN_EINVAL, "NULL tree");
        if (trees[i]->n_trees != 1) return knn::fail(KNN_EINVAL, "forests are not served");
        if (trees[i]->device != trees[0]->device) return knn::fail(KNN_EINVAL, "trees on two devices");
        if (trees[i]->depth + 1 > knn::kWave)
            return knn::fail(KNN_EINVAL, "a tree deeper than 63 levels cannot be served");
    }
    auto* s = new knn_server();
    s->trees.assign(trees, trees + ntrees);
    s->device = trees[0]->device;
    s->budget = q.hbm_budget_bytes ? q.hbm_budget_bytes : (int64_t(4) << 30);
    s->slot_max = std::min<int64_t>(q.slot_max_queries, kSlotMaxQueries);
    const int ns = q.streams ? q.streams : 4;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    auto undo = [&](const char* what) {
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        for (auto& k : s->slotk) {
            if (k.stream) (void)hipStreamDestroy(k.stream);
            if (k.ended) (void)hipEventDestroy(k.ended);
            if (k.host) (void)hipHostFree(k.host);
            if (k.dev) (void)hipFree(k.dev);
        }
        (void)hipSetDevice(prev);
        delete s;
        return knn::fail(KNN_EDEVICE, what);
    };
    for (int i = 0; i < ns; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return undo("stream creation failed");
        s->streams.push_back(st);
    }
    s->busy.assign(ns, false);
    if (s->slot_max > 0) {
        int cus = 0, khz = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess ||
            cus < 1 || khz < 1)
            return undo("device attributes unavailable");
        s->slot_blocks = cus * (q.slot_workgroups_per_cu ? q.slot_workgroups_per_cu : kSlotWgPerCu);
        s->idle_ticks = (uint64_t)khz * (q.slot_idle_us ? q.slot_idle_us : kSlotIdleUs) / 1000;
        s->life_ticks = (uint64_t)khz * kSlotLifeMs;
        s->watchdog_ticks = (uint64_t)khz * kSlotWatchdogMs;
        s->slotk.resize(ntrees);
        for (auto& k : s->slotk) {
            void* h = nullptr;
            if (hipHostMalloc(&h, sizeof(PHost), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
                return undo("pinned host allocation failed");
            std::memset(h, 0, sizeof(PHost));
            k.host = static_cast<PHost*>(h);
            if (hipMalloc(&k.dev, sizeof(PDev)) != hipSuccess) return undo("device allocation failed");
            if (hipMemset(k.dev, 0, sizeof(PDev)) != hipSuccess ||
                hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&k.ended, hipEventDisableTiming) != hipSuccess)
                return undo("slot kernel set-up failed");
        }
    }
    (void)hipSetDevice(prev);
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return KNN_OK;
}

int knn_server_create(const knn_tree* const* trees, int32_t ntrees, int64_t hbm_budget_bytes,
                      int32_t streams, knn_server** out)
{
    const knn_server_params p{hbm_budget_bytes, streams, 0, 0, 0};
    return knn_server_create_ex(trees, ntrees, &p, out);
}

int knn_server_submit(knn_server* s, int32_t tree, const float* queries, int64_t m, int32_t k,
                      const int32_t* self_ids, int32_t* out_idx, float* out_dist2,
                      int64_t* ticket)
{
    if (!s || !ticket) return knn::fail(KNN_EINVAL, "NULL argument");
    *ticket = 0;
    if (tree < 0 || tree >= (int32_t)s->trees.size()) return knn::fail(KNN_EINVAL, "bad tree");
    if (m < 1 || m > kMaxBatchQueries) return knn::fail(KNN_EINVAL, "m must be in [1, 2^18]");
    if (k < 1 || k > KNN_MAX_K) return knn::fail(KNN_EINVAL, "k must be in [1, 64]");
    if (!queries || !out_idx || !out_dist2) return knn::fail(KNN_EINVAL, "NULL buffer");
    auto* r = new Request();
    r->tree = tree;
    r->q = queries;
    r->m = m;
    r->k = k;
    r->self = self_ids;
    r->oi = out_idx;
    r->od = out_dist2;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return knn::fail(KNN_EINVAL, "server is shutting down");
        }
        r->ticket = s->next_ticket++;
        r->t_submit = now_ms();
        s->reqs[r->ticket] = r;
        s->pending.push_back(r);
        ++s->n_requests;
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return KNN_OK;
}

int knn_server_wait(knn_server* s, int64_t ticket, double* latency_ms)
{
    if (!s) return knn::fail(KNN_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return knn::fail(KNN_EINVAL, "unknown ticket");
    Request* r = it->second;
    s->cv_done.wait(lk, [r] { return r->status != 1; });
    const int st = r->status;
    if (latency_ms) *latency_ms = r->t_done - r->t_submit;
    s->reqs.erase(it);
    delete r;
    return st == KNN_OK ? KNN_OK : knn::fail(st, "the request's batch failed on the device");
}

int knn_server_stats(knn_server* s, int64_t* out /* [KNN_SERVER_STATS] */)
{
    if (!s || !out) return knn::fail(KNN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->n_requests;
    out[1] = s->n_batches;
    out[2] = s->n_queries;
    out[3] = s->peak_bytes;
    out[4] = s->max_reqs_per_batch;
    out[5] = s->peak_inflight;
    out[6] = s->max_k_kinds;
    out[7] = s->joined_running;
    out[8] = s->n_slot_requests;
    out[9] = s->n_slot_launches;
    return KNN_OK;
}

int knn_server_destroy(knn_server* s)
{
    if (!s) return KNN_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto& k : s->slotk) {  // nothing is in flight: a launch still waiting ends at once
        __atomic_store_n(&k.host->stop, uint64_t(1), __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(k.stream);
        (void)hipStreamDestroy(k.stream);
        (void)hipEventDestroy(k.ended);
        (void)hipHostFree(k.host);
        (void)hipFree(k.dev);
    }
    (void)hipSetDevice(prev);
    for (auto& kv : s->reqs) delete kv.second;  // tickets never waited for
    delete s;
    return KNN_OK;
}

}  // extern "C"
