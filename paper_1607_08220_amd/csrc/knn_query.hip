// Batched exact k-NN queries on gfx950 (Algorithm 1, Sections III-B/III-C of
// arXiv 1607.08220).
//
// One lane per query.  Algorithm 1 keeps an explicit stack of (node, bound);
// here every node stores its parent, so the traversal needs no stack: a lane
// remembers only the node it is at and the node it came from.  Arriving at a
// node from above, the lane tests the node's tight box bound against r' (the
// k-th best distance so far) and either scans it (leaf), descends to the near
// child, or goes back up.  Coming back up from the near child it tests the
// split-plane bound of the far child and descends there if it may hold a
// closer point; coming back from the far child it goes up again.  This visits
// the same nodes as Algorithm 1 with the near child pushed last, with the
// bounds re-tested against the current r'.
//
// Queries are first grouped by the leaf that contains them (k_locate +
// counting sort), and a lane starts at its query's home leaf: the leaf is
// scanned first, which tightens r' immediately (the near-first order of the
// paper), and adjacent lanes walk nearly the same nodes, so loads coalesce.
//
// The heap H is a sorted register array of KC >= k entries; the lowest KC-k
// slots hold (-inf) sentinels so the top k slots behave as a k-entry bounded
// max-heap with its maximum in slot KC-1.  Empty slots hold (r2, -1): a point
// enters iff (D, i) < (top D, top i), which for an empty slot means D < r2.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "knn_internal.h"

namespace knn {
namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;  // accelerator complex dies of an MI355X, each with its own L2

// q[dim] as a chain of selects.  The empty asm keeps the compiler from
// turning the chain back into a dynamically indexed array (which it would
// place in LDS).
template <int D>
__device__ inline float select_dim(const float (&q)[D], int dim)
{
    float v = q[0];
#pragma unroll
    for (int t = 1; t < D; ++t) {
        asm volatile("" : "+v"(v));
        v = dim == t ? q[t] : v;
    }
    return v;
}

// The node's box [lo, hi] (2D floats, 8-byte aligned), loaded without branches.
template <int D>
__device__ inline void load_box(const float* __restrict__ bb, float (&b)[2 * D])
{
#pragma unroll
    for (int t = 0; t < 2 * D; t += 2) {
        const float2 v = *reinterpret_cast<const float2*>(bb + t);
        b[t] = v.x;
        b[t + 1] = v.y;
    }
}

// Sum over dimensions, left to right, of the squared offset of q from the
// box [lo, hi]: max(lo - q, q - hi, 0) per dimension.  Rounding is monotone,
// so this is <= the FP32 distance from q to every point in the box.
template <int D>
__device__ inline float box_bound(const float (&q)[D], const float (&b)[2 * D])
{
    float acc = 0.0f;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const float o = fmaxf(fmaxf(b[t] - q[t], q[t] - b[D + t]), 0.0f);
        const float sq = o * o;
        acc = t == 0 ? sq : acc + sq;
    }
    return acc;
}

template <int D>
__device__ inline void load_row(const float* __restrict__ row, float (&x)[D + 1])
{
    if constexpr ((D + 1) % 4 == 0) {
#pragma unroll
        for (int t = 0; t < D + 1; t += 4) {
            const float4 v = *reinterpret_cast<const float4*>(row + t);
            x[t] = v.x; x[t + 1] = v.y; x[t + 2] = v.z; x[t + 3] = v.w;
        }
    } else if constexpr ((D + 1) % 2 == 0) {
#pragma unroll
        for (int t = 0; t < D + 1; t += 2) {
            const float2 v = *reinterpret_cast<const float2*>(row + t);
            x[t] = v.x; x[t + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int t = 0; t < D + 1; ++t) x[t] = row[t];
    }
}

__device__ inline bool key_less(float d, int i, float td, int ti)
{
    return d < td || (d == td && i < ti);
}

template <int KC>
__device__ inline void heap_insert(float (&hd)[KC], int (&hi)[KC], float D, int I)
{
#pragma unroll
    for (int p = KC - 1; p >= 1; --p) {
        const bool below_prev = key_less(D, I, hd[p - 1], hi[p - 1]);
        const bool below_cur = key_less(D, I, hd[p], hi[p]);
        const float nd = below_prev ? hd[p - 1] : (below_cur ? D : hd[p]);
        const int ni = below_prev ? hi[p - 1] : (below_cur ? I : hi[p]);
        hd[p] = nd;
        hi[p] = ni;
    }
    if (key_less(D, I, hd[0], hi[0])) {
        hd[0] = D;
        hi[0] = I;
    }
}

// STATS adds visit counters (nodes entered from above, leaves scanned, points
// scanned) summed per wavefront into stats[0..2]; the timed kernel has none.
template <int D, int KC, bool STATS>
__global__ __launch_bounds__(kBlock) void k_traverse(
    const NodeRec* __restrict__ nodes, const float* __restrict__ bbox,
    const float* __restrict__ pts, const float* __restrict__ queries,
    const int32_t* __restrict__ order, const int32_t* __restrict__ home,
    const int32_t* __restrict__ self_ids, int64_t m, int k, float r2,
    int32_t* __restrict__ out_idx, float* __restrict__ out_d2,
    unsigned long long* __restrict__ stats)
{
    // XCD-aware order: consecutive blocks are dispatched to the 8 XCDs in
    // turn, so block b takes chunk (b % 8) * per + b / 8 -- each XCD then
    // walks one contiguous range of the grouped queries and their leaves
    // stay in its own L2.  The grid is a multiple of 8; extra blocks exit.
    const int64_t per = gridDim.x / kXcds;
    const int64_t blk = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int64_t slot = blk * blockDim.x + threadIdx.x;
    unsigned long long n_enter = 0, n_leaf = 0, n_pts = 0;
    if (slot < m) {  // every lane meets the counter sums below
    const int64_t qid = order ? order[slot] : slot;
    float q[D];
#pragma unroll
    for (int t = 0; t < D; ++t) q[t] = queries[qid * D + t];
    const int32_t self = self_ids ? self_ids[qid] : -1;
    float hd[KC];
    int hi[KC];
    const int pad = KC - k;
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        hd[j] = j < pad ? -INFINITY : r2;
        hi[j] = j < pad ? INT_MIN : -1;
    }
    int cur = home ? home[slot] : 0;
    int from = -1;  // -1: arrived from the parent; otherwise the child we came from
    // The record and box of `cur` are loaded at the end of the step that moves
    // there, together, so one memory latency is exposed per step.
    NodeRec r = nodes[cur];
    float bb[2 * D];
    load_box<D>(bbox + (int64_t)cur * (2 * D), bb);
    while (cur >= 0) {
        int lstart = 0, lcnt = 0;
        while (cur >= 0) {
            int next, nfrom;
            bool scan = false;
            if (from < 0) {
                if constexpr (STATS) ++n_enter;
                const float b = box_bound<D>(q, bb);
                if (b > hd[KC - 1]) {  // no point of this node can enter H
                    next = r.parent;
                    nfrom = cur;
                } else if (r.dim < 0) {  // leaf: scan it below, then return to the parent
                    lstart = r.a;
                    lcnt = -r.dim;
                    next = r.parent;
                    nfrom = cur;
                    scan = true;
                } else {
                    const float qd = select_dim<D>(q, r.dim);
                    next = qd < r.split ? r.a : r.a + 1;  // near child first
                    nfrom = -1;
                }
            } else {
                const float qd = select_dim<D>(q, r.dim);
                const bool left_near = qd < r.split;
                const int near = left_near ? r.a : r.a + 1;
                const float o = left_near ? r.split - qd : qd - r.split;
                if (from == near && o * o <= hd[KC - 1]) {  // split-plane bound of the far child
                    next = left_near ? r.a + 1 : r.a;
                    nfrom = -1;
                } else {
                    next = r.parent;
                    nfrom = cur;
                }
            }
            cur = next;
            from = nfrom;
            if (cur >= 0) {
                r = nodes[cur];
                load_box<D>(bbox + (int64_t)cur * (2 * D), bb);
            }
            if (scan) break;
        }
        if constexpr (STATS) {
            n_leaf += lcnt > 0;
            n_pts += lcnt;
        }
        // bucket rows are loaded B at a time so that their latencies overlap
        constexpr int B = D <= 4 ? 8 : 4;
        for (int j0 = 0; j0 < lcnt; j0 += B) {
            float x[B][D + 1];
            // unconditional loads (the last row repeats past the end) so all B
            // are in flight at once; only the arithmetic below is masked
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = j0 + b < lcnt ? j0 + b : lcnt - 1;
                load_row<D>(pts + (int64_t)(lstart + j) * (D + 1), x[b]);
            }
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (j0 + b < lcnt) {
                    const float t0 = q[0] - x[b][0];
                    float acc = t0 * t0;
#pragma unroll
                    for (int t = 1; t < D; ++t) {
                        const float u = q[t] - x[b][t];
                        const float sq = u * u;
                        acc = acc + sq;
                    }
                    if (acc <= hd[KC - 1]) {
                        const int id = __float_as_int(x[b][D]);
                        if (id != self && key_less(acc, id, hd[KC - 1], hi[KC - 1]))
                            heap_insert<KC>(hd, hi, acc, id);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        if (j >= pad) {
            const int64_t o = qid * k + (j - pad);
            const int id = hi[j];
            out_idx[o] = id;
            out_d2[o] = id < 0 ? INFINITY : hd[j];
        }
    }
    }  // slot < m
    if constexpr (STATS) {
        for (int o = 32; o > 0; o >>= 1) {
            n_enter += __shfl_xor(n_enter, o);
            n_leaf += __shfl_xor(n_leaf, o);
            n_pts += __shfl_xor(n_pts, o);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&stats[0], n_enter);
            atomicAdd(&stats[1], n_leaf);
            atomicAdd(&stats[2], n_pts);
        }
    }
}

// Home leaf of every query: descend with the near-child rule (x < split
// left).  Queries are grouped by key = (first packed position of the home
// leaf) >> shift: buckets are contiguous in packed order, so key order is the
// tree's spatial order.
template <int D>
__global__ __launch_bounds__(kBlock) void k_locate(const NodeRec* __restrict__ nodes,
                                                   const float* __restrict__ queries, int64_t m,
                                                   int shift, int32_t* __restrict__ home,
                                                   uint32_t* __restrict__ cnt)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    float q[D];
#pragma unroll
    for (int t = 0; t < D; ++t) q[t] = queries[i * D + t];
    int cur = 0;
    NodeRec r = nodes[0];
    while (r.dim >= 0) {
        cur = select_dim<D>(q, r.dim) < r.split ? r.a : r.a + 1;
        r = nodes[cur];
    }
    home[i] = cur;
    atomicAdd(&cnt[r.a >> shift], 1u);
}

__global__ __launch_bounds__(kBlock) void k_group(const NodeRec* __restrict__ nodes,
                                                  const int32_t* __restrict__ home, int64_t m,
                                                  int shift, uint32_t* __restrict__ offs,
                                                  int32_t* __restrict__ order,
                                                  int32_t* __restrict__ shome)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int h = home[i];
    const uint32_t p = atomicAdd(&offs[nodes[h].a >> shift], 1u);
    order[p] = (int32_t)i;
    shome[p] = h;
}

// Exclusive scan of uint32 in place: per-block scan of 4096 values, a scan
// of the block sums, then the block offsets are added.
constexpr int kScanItems = 16;
constexpr int kScanChunk = kBlock * kScanItems;

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

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t* __restrict__ a, int64_t len,
                                                     const uint32_t* __restrict__ bsum)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < len) a[i] += bsum[i / kScanChunk];
}

using TraverseFn = void (*)(const NodeRec*, const float*, const float*, const float*,
                            const int32_t*, const int32_t*, const int32_t*, int64_t, int, float,
                            int32_t*, float*, unsigned long long*);
using LocateFn = void (*)(const NodeRec*, const float*, int64_t, int, int32_t*, uint32_t*);

template <int D, bool STATS>
TraverseFn pick_traverse(int k)
{
    if (k <= 4) return k_traverse<D, 4, STATS>;
    if (k <= 8) return k_traverse<D, 8, STATS>;
    if (k <= 16) return k_traverse<D, 16, STATS>;
    if (k <= 32) return k_traverse<D, 32, STATS>;
    return k_traverse<D, 64, STATS>;
}

TraverseFn traverse_for(int d, int k, bool stats)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return stats ? pick_traverse<DD, true>(k) : pick_traverse<DD, false>(k);
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

}  // namespace

int query_tree(const knn_tree* t, const float* queries, int64_t m, int32_t k,
               const int32_t* self_ids, float r2, int32_t order, int32_t* out_idx,
               float* out_d2, unsigned long long* stats, hipStream_t st)
{
    const int d = t->d;
    TraverseFn tf = traverse_for(d, k, stats != nullptr);
    LocateFn lf = locate_for(d);
    if (!tf || !lf) return fail(KNN_EINVAL, "unsupported dimension");
    prof_mark(st, 5);
    const unsigned grid = (unsigned)((m + kBlock - 1) / kBlock);
    const unsigned tgrid = (unsigned)((grid + kXcds - 1) / kXcds * kXcds);  // multiple of 8
    if (order == 1) {
        prof_mark(st, 6);
        prof_mark(st, 7);
        hipLaunchKernelGGL(tf, dim3(tgrid), dim3(kBlock), 0, st, t->nodes, t->bbox, t->pts,
                           queries, nullptr, nullptr, self_ids, m, k, r2, out_idx, out_d2, stats);
        KNN_HIP(hipGetLastError());
        prof_mark(st, 8);
        return KNN_OK;
    }
    // key range: packed positions >> shift, at most 2^22 buckets
    int shift = 0;
    while ((t->n >> shift) > (int64_t(1) << 22)) ++shift;
    const int64_t N = (t->n >> shift) + 1;
    const int64_t nsb = (N + kScanChunk - 1) / kScanChunk;
    // workspace: home[m], order[m], shome[m], cnt[N], block sums[nsb]
    const size_t bytes = sizeof(int32_t) * 3 * (size_t)m + sizeof(uint32_t) * (size_t)(N + nsb);
    StreamBuf ws;
    ws.s = st;
    KNN_HIP(hipMallocAsync(&ws.p, bytes, st));
    int32_t* home = static_cast<int32_t*>(ws.p);
    int32_t* ord = home + m;
    int32_t* shome = ord + m;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(shome + m);
    uint32_t* bsum = cnt + N;
    KNN_HIP(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * N, st));
    hipLaunchKernelGGL(lf, dim3(grid), dim3(kBlock), 0, st, t->nodes, queries, m, shift, home, cnt);
    KNN_HIP(hipGetLastError());
    prof_mark(st, 6);
    k_scan_local<<<(unsigned)nsb, kBlock, 0, st>>>(cnt, N, bsum);
    k_scan_sums<<<1, kBlock, 0, st>>>(bsum, nsb);
    k_scan_add<<<(unsigned)((N + kBlock - 1) / kBlock), kBlock, 0, st>>>(cnt, N, bsum);
    k_group<<<grid, kBlock, 0, st>>>(t->nodes, home, m, shift, cnt, ord, shome);
    KNN_HIP(hipGetLastError());
    prof_mark(st, 7);
    hipLaunchKernelGGL(tf, dim3(tgrid), dim3(kBlock), 0, st, t->nodes, t->bbox, t->pts, queries,
                       ord, shome, self_ids, m, k, r2, out_idx, out_d2, stats);
    KNN_HIP(hipGetLastError());
    prof_mark(st, 8);
    return KNN_OK;
}

}  // namespace knn
