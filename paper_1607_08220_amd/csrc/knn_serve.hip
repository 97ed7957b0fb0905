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
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "knn_internal.h"

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

struct knn_server {
    std::vector<const knn_tree*> trees;
    int device = 0;
    int64_t budget = 0;
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

// Device bytes a batch needs: staging for its queries, self ids, per-query
// k and output offsets, and results, plus the grouping workspace of the
// query path when it runs.
size_t batch_bytes(const knn_tree* t, int64_t total, int64_t outputs)
{
    size_t b = (size_t)total * (sizeof(float) * t->d + sizeof(int32_t) * 2 + sizeof(int64_t)) +
               (size_t)outputs * 8;
    if (total >= kGroupMin) {
        int shift = 0;
        while ((t->n >> shift) > (int64_t(1) << 22)) ++shift;
        b += sizeof(uint32_t) * ((size_t)(t->n >> shift) + 2 + 4096) + sizeof(int32_t) * 3 * total;
    }
    return b;
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
    KNN_HIP(hipMallocAsync(&b.mem, b_qout + b_q + 2 * b_i + 2 * b_o, b.stream));
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
    knn::QuerySpec qs;
    qs.queries = q;
    qs.m = total;
    qs.k = b.kmax;
    qs.qk = qk;
    qs.qout = qout;
    qs.self_ids = self;
    qs.order = total >= kGroupMin ? 0 : 1;
    qs.batch = knn::kDefaultLeafBatch;
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

void worker_loop(knn_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        // retire the batches whose work has completed
        bool retired = false;
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
        while (!s->pending.empty()) {
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
                if (r->tree == head->tree && (b.reqs.empty() || total + r->m <= kMaxBatchQueries)) {
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
            b.bytes = batch_bytes(t, total, b.outputs);
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
        if (s->stop && s->pending.empty() && s->inflight.empty()) break;
        if (s->inflight.empty()) {
            s->cv_work.wait(lk, [s] { return s->stop || !s->pending.empty(); });
        } else {
            // poll the events in flight; new requests wake the loop as well
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

extern "C" {

int knn_server_create(const knn_tree* const* trees, int32_t ntrees, int64_t hbm_budget_bytes,
                      int32_t streams, knn_server** out)
{
    if (!out) return knn::fail(KNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!trees || ntrees < 1) return knn::fail(KNN_EINVAL, "no trees");
    if (hbm_budget_bytes < 0 || streams < 0 || streams > 64)
        return knn::fail(KNN_EINVAL, "budget must be >= 0 and streams in [0, 64]");
    for (int32_t i = 0; i < ntrees; ++i) {
        if (!trees[i]) return knn::fail(KNN_EINVAL, "NULL tree");
        if (trees[i]->n_trees != 1) return knn::fail(KNN_EINVAL, "forests are not served");
        if (trees[i]->device != trees[0]->device) return knn::fail(KNN_EINVAL, "trees on two devices");
    }
    auto* s = new knn_server();
    s->trees.assign(trees, trees + ntrees);
    s->device = trees[0]->device;
    s->budget = hbm_budget_bytes ? hbm_budget_bytes : (int64_t(4) << 30);
    const int ns = streams ? streams : 4;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (int i = 0; i < ns; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            (void)hipSetDevice(prev);
            delete s;
            return knn::fail(KNN_EDEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    s->busy.assign(ns, false);
    (void)hipSetDevice(prev);
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return KNN_OK;
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
    (void)hipSetDevice(prev);
    for (auto& kv : s->reqs) delete kv.second;  // tickets never waited for
    delete s;
    return KNN_OK;
}

}  // extern "C"
