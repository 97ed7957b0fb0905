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
// bounds re-tested against the current r'.  For deep high-dimensional walks
// k_traverse_stack keeps Algorithm 1's explicit stack instead (in LDS), and
// batches too small to fill the device with one lane per query are answered
// by k_traverse_wave, one wavefront per query.
//
// Queries are first grouped by the leaf that contains them (k_locate +
// counting sort), and a lane starts at its query's home leaf: the leaf is
// scanned first, which tightens r' immediately (the near-first order of the
// paper), and adjacent lanes walk nearly the same nodes, so loads coalesce.
//
// The heap H is a sorted register array of KC >= k keys (D, i); the lowest
// KC-k slots hold the key 0, below every point, so the top k slots behave as
// a k-entry bounded max-heap with its maximum in slot KC-1.  Empty slots hold
// (r2, 0): a point enters iff (D, i) < the top key, which for an empty slot
// means D < r2 (and for r2 <= 0, never).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "knn_internal.h"

namespace knn {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcds = 8;                      // accelerator complex dies of an MI355X, each with its own L2
constexpr size_t kMaxStackLds = 160 * 1024;  // LDS of one workgroup on gfx950
constexpr int kStackMinDim = 5;               // default: explicit stack from 5 dimensions
constexpr int64_t kWaveQueriesMax = 16384;    // default: one wavefront per query up to this batch

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

// 1 in the lowest-numbered active lane of the wavefront, else 0.
__device__ inline unsigned first_active_lane()
{
    const unsigned long long ex = __builtin_amdgcn_read_exec();
    return __lane_id() == (unsigned)__builtin_ctzll(ex);
}

// FP32 squared distance: separate multiply and add, summed left to right.
template <int D>
__device__ inline float distance(const float (&q)[D], const float (&x)[D + 1])
{
    const float t0 = q[0] - x[0];
    float acc = t0 * t0;
#pragma unroll
    for (int t = 1; t < D; ++t) {
        const float u = q[t] - x[t];
        const float sq = u * u;
        acc = acc + sq;
    }
    return acc;
}

// Heap entries are 64-bit keys: the FP32 distance bits in the high word (a
// non-negative float orders like its bit pattern) and the point index in the
// low word, so unsigned key order is the (D, i) order.
__device__ inline uint64_t make_key(float d, int i)
{
    return ((uint64_t)__float_as_uint(d) << 32) | (uint32_t)i;
}

__device__ inline float key_dist(uint64_t key) { return __uint_as_float((uint32_t)(key >> 32)); }

// Insert key into the ascending array h, dropping h[KC-1]; the caller has
// checked key < h[KC-1].  Branch-free: one compare and two selects per slot.
template <int KC>
__device__ inline void heap_insert(uint64_t (&h)[KC], uint64_t key)
{
    bool below = true;  // key < h[p]
#pragma unroll
    for (int p = KC - 1; p >= 1; --p) {
        const bool below_prev = key < h[p - 1];
        h[p] = below_prev ? h[p - 1] : (below ? key : h[p]);
        below = below_prev;
    }
    h[0] = below ? key : h[0];
}

// True if the ball around q of squared radius thr lies strictly inside the
// box [lo, hi]: per dimension m = min(q - lo, hi - q) > 0 and m*m > thr.  A
// point x outside the box differs from q in some dimension by at least m, so
// (rounding being monotone) its FP32 distance is >= fl(m*m) > thr and it
// cannot enter H.
template <int D>
__device__ inline bool ball_inside(const float (&q)[D], const float (&b)[2 * D], float thr)
{
    bool in = true;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const float mt = fminf(q[t] - b[t], b[D + t] - q[t]);
        in = in && mt > 0.0f && mt * mt > thr;
    }
    return in;
}

}  // namespace

// Arguments of one traversal launch.  Per-query arrays are indexed by the
// query's position in `queries`; NULL selects the scalar beside it.
struct TravArgs {
    const NodeRec* nodes;
    const float* bbox;
    const float* pts;
    const float* queries;   // [m][D]
    const int32_t* order;   // slot -> query (NULL: identity)
    const int32_t* home;    // slot -> home leaf (NULL: start at the query's root)
    const int32_t* root;    // per-query root node (a forest's tree), else node 0
    int32_t n_roots;        // valid root ids: [0, n_roots)
    unsigned long long* bad;  // count of queries whose root id is out of range
    const int32_t* self_ids;
    const float* r2s;       // per-query squared radius, else r2
    const int32_t* qk;      // per-query k (<= the kernel's capacity), else k
    const int64_t* qout;    // per-query first output element, else query * k
    float r2;
    int k;
    int batch;
    int64_t m;
    int32_t* out_idx;
    float* out_d2;
    unsigned long long* stats;
};

namespace {

// Root node of query qid: its tree's root (tree t of a forest is node t), or
// -1 when the caller's tree id is out of range -- such a query visits no node,
// is answered with padding rows, and is counted in A.bad.
__device__ inline int query_root(const TravArgs& A, int64_t qid)
{
    if (!A.root) return 0;
    const int r = A.root[qid];
    if ((unsigned)r < (unsigned)A.n_roots) return r;
    atomicAdd(A.bad, 1ull);
    return -1;
}

// STATS adds visit counters summed per wavefront into stats[0..8]: per lane
// (nodes entered from above, leaves scanned, points scanned, traversal steps,
// heap inserts) and per wavefront (traversal-loop iterations, bucket-row
// batches, leaf rounds, heap-insert executions); the timed kernel has none.
// The wavefront counts are taken by its first active lane, so their ratio to
// the lane counts measures divergence.  RB bucket rows are loaded per batch.
//
// Lanes walk the tree until they reach a bucket to scan; a lane holding a
// bucket pauses, and the wavefront scans once at least `batch` of every 64 of
// its unfinished lanes hold one (or no lane can walk on).  Waiting for every
// lane (batch = 64) leaves most lanes idle while the slowest one walks;
// scanning for a single lane wastes the scan loop.  The result does not depend
// on `batch`.
//
// A lane whose search ball lies inside the tight box of the node it is
// leaving upwards stops: every point outside that box is farther than r'.
template <int D, int KC, bool STATS, int RB>
__global__ __launch_bounds__(kBlock) void k_traverse(TravArgs A)
{
    const NodeRec* __restrict__ nodes = A.nodes;
    const float* __restrict__ bbox = A.bbox;
    const float* __restrict__ pts = A.pts;
    const float* __restrict__ queries = A.queries;
    const int32_t* __restrict__ order = A.order;
    const int32_t* __restrict__ home = A.home;
    const int32_t* __restrict__ self_ids = A.self_ids;
    const int64_t m = A.m;
    const int batch = A.batch;
    unsigned long long* __restrict__ stats = A.stats;
    // XCD-aware order: consecutive blocks are dispatched to the 8 XCDs in
    // turn, so block b takes chunk (b % 8) * per + b / 8 -- each XCD then
    // walks one contiguous range of the grouped queries and their leaves
    // stay in its own L2.  The grid is a multiple of 8; extra blocks exit.
    const int64_t per = gridDim.x / kXcds;
    const int64_t blk = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int64_t slot = blk * blockDim.x + threadIdx.x;
    unsigned long long n_enter = 0, n_leaf = 0, n_pts = 0, n_step = 0, n_ins = 0;
    unsigned long long w_step = 0, w_rows = 0, w_round = 0, w_ins = 0;
    if (slot < m) {  // every lane meets the counter sums below
    const int64_t qid = order ? order[slot] : slot;
    float q[D];
#pragma unroll
    for (int t = 0; t < D; ++t) q[t] = queries[qid * D + t];
    const int32_t self = self_ids ? self_ids[qid] : -1;
    uint64_t h[KC];
    const int k = A.qk ? A.qk[qid] : A.k;
    const int pad = KC - k;
    const float r2 = A.r2s ? A.r2s[qid] : A.r2;
    const uint64_t empty = r2 > 0.0f ? make_key(r2, 0) : 0;
#pragma unroll
    for (int j = 0; j < KC; ++j) h[j] = j < pad ? 0 : empty;
    const int root = query_root(A, qid);
    int cur = root < 0 ? -1 : (home ? home[slot] : root);
    int from = -1;  // -1: arrived from the parent; otherwise the child we came from
    // The record and box of `cur` are loaded at the end of the step that moves
    // there, together, so one memory latency is exposed per step.
    NodeRec r{};
    float bb[2 * D];
    if (cur >= 0) {
        r = nodes[cur];
        load_box<D>(bbox + (int64_t)cur * (2 * D), bb);
    }
    int lstart = 0, lcnt = 0;  // the bucket waiting to be scanned (lcnt > 0)
    while (true) {
        if constexpr (STATS) w_round += first_active_lane();
        while (true) {
            const bool walking = cur >= 0 && lcnt == 0;
            const unsigned long long wb = __ballot(walking);
            if (wb == 0) break;
            const int held = __popcll(__ballot(lcnt > 0));
            if (held * 64 >= batch * (held + __popcll(wb))) break;
            if (walking) {
                if constexpr (STATS) {
                    ++n_step;
                    w_step += first_active_lane();
                }
                const float thr = key_dist(h[KC - 1]);
                int next, nfrom;
                bool up = false;  // leaving upwards: stop if the ball lies inside the box
                if (from < 0) {
                    if constexpr (STATS) ++n_enter;
                    const float b = box_bound<D>(q, bb);
                    if (b > thr) {  // no point of this node can enter H
                        next = r.parent;
                        nfrom = cur;
                    } else if (r.dim < 0) {  // leaf: scan it, then return to the parent
                        lstart = r.a;
                        lcnt = -r.dim;
                        next = r.parent;
                        nfrom = cur;
                        up = true;
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
                    if (from == near && o * o <= thr) {  // split-plane bound of the far child
                        next = left_near ? r.a + 1 : r.a;
                        nfrom = -1;
                    } else {
                        next = r.parent;
                        nfrom = cur;
                        up = true;
                    }
                }
                if (up && ball_inside<D>(q, bb, thr)) next = -1;
                cur = next;
                from = nfrom;
                if (cur >= 0) {
                    r = nodes[cur];
                    load_box<D>(bbox + (int64_t)cur * (2 * D), bb);
                }
            }
        }
        if (__ballot(lcnt > 0) == 0) break;  // no lane walks and none holds a bucket
        if constexpr (STATS) {
            n_leaf += lcnt > 0;
            n_pts += lcnt;
        }
        // Bucket rows are loaded B at a time so that their latencies overlap;
        // rows past the bucket (the next bucket's, or the zero rows after the
        // last one) are loaded too, and only the arithmetic is masked.
        constexpr int B = RB;
        static_assert(B <= kRowPad, "row batches must fit in the padding rows");
        const float* row0 = pts + (int64_t)lstart * (D + 1);
        if (__ballot(lcnt > 0 && h[KC - 1] == empty) != 0) {
            // Some heap is still filling, so most rows enter: insert each row
            // as soon as its distance is known.
            for (int j0 = 0; j0 < lcnt; j0 += B) {
                if constexpr (STATS) w_rows += first_active_lane();
                float x[B][D + 1];
#pragma unroll
                for (int b = 0; b < B; ++b) load_row<D>(row0 + (j0 + b) * (D + 1), x[b]);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int id = __float_as_int(x[b][D]);
                    const uint64_t key = make_key(distance<D>(q, x[b]), id);
                    if (j0 + b < lcnt && key < h[KC - 1] && id != self) {
                        if constexpr (STATS) {
                            ++n_ins;
                            w_ins += first_active_lane();
                        }
                        heap_insert<KC>(h, key);
                    }
                }
            }
        } else {
            // Every heap is full and few rows enter: mark the rows of a batch
            // below the top, then insert only those, so a wavefront runs as
            // many inserts as its busiest lane needs instead of one per row.
            for (int j0 = 0; j0 < lcnt; j0 += B) {
                if constexpr (STATS) w_rows += first_active_lane();
                float x[B][D + 1];
#pragma unroll
                for (int b = 0; b < B; ++b) load_row<D>(row0 + (j0 + b) * (D + 1), x[b]);
                uint64_t keys[B];
                unsigned cand = 0;
                const uint64_t top = h[KC - 1];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int id = __float_as_int(x[b][D]);
                    keys[b] = make_key(distance<D>(q, x[b]), id);
                    if (j0 + b < lcnt && keys[b] < top && id != self) cand |= 1u << b;
                }
                while (cand) {
                    const int j = __builtin_ctz(cand);
                    cand &= cand - 1;
                    uint64_t key = keys[0];
#pragma unroll
                    for (int b = 1; b < B; ++b) key = j == b ? keys[b] : key;
                    if (key < h[KC - 1]) {
                        if constexpr (STATS) {
                            ++n_ins;
                            w_ins += first_active_lane();
                        }
                        heap_insert<KC>(h, key);
                    }
                }
            }
        }
        lcnt = 0;
    }
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        if (j >= pad) {
            const int64_t o = (A.qout ? A.qout[qid] : qid * k) + (j - pad);
            const bool none = h[j] == empty;
            A.out_idx[o] = none ? -1 : (int)(uint32_t)h[j];
            A.out_d2[o] = none ? INFINITY : key_dist(h[j]);
        }
    }
    }  // slot < m
    if constexpr (STATS) {
        unsigned long long c[9] = {n_enter, n_leaf, n_pts, n_step, n_ins,
                                   w_step, w_rows, w_round, w_ins};
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            for (int o = 32; o > 0; o >>= 1) c[j] += __shfl_xor(c[j], o);
            if ((threadIdx.x & 63) == 0) atomicAdd(&stats[j], c[j]);
        }
    }
}

// Algorithm 1 with its explicit stack, for deep walks (high dimensions):
// each lane starts at its query's root and keeps the far children it has
// still to visit, with their split-plane bounds, in a stack in LDS (at most
// one entry per level of the path, so depth + 1 entries).  A popped entry
// whose bound exceeds r' is dropped without touching HBM, where the
// stack-free walk pays one dependent load per ancestor it climbs back
// through.  Bucket scans, the heap and the wavefront vote are those of
// k_traverse.
constexpr int kPopAfterScan = -2;

template <int D, int KC, bool STATS, int RB>
__global__ __launch_bounds__(kBlock) void k_traverse_stack(TravArgs A, int sdepth)
{
    extern __shared__ int2 stk[];  // [sdepth][kBlock]: entry j of lane t at j * kBlock + t
    const NodeRec* __restrict__ nodes = A.nodes;
    const float* __restrict__ bbox = A.bbox;
    const float* __restrict__ pts = A.pts;
    const int64_t m = A.m;
    const int batch = A.batch;
    const int64_t per = gridDim.x / kXcds;
    const int64_t blk = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int64_t slot = blk * blockDim.x + threadIdx.x;
    unsigned long long n_enter = 0, n_leaf = 0, n_pts = 0, n_step = 0, n_ins = 0;
    unsigned long long w_step = 0, w_rows = 0, w_round = 0, w_ins = 0;
    if (slot < m) {  // every lane meets the counter sums below
    const int64_t qid = A.order ? A.order[slot] : slot;
    float q[D];
#pragma unroll
    for (int t = 0; t < D; ++t) q[t] = A.queries[qid * D + t];
    const int32_t self = A.self_ids ? A.self_ids[qid] : -1;
    uint64_t h[KC];
    const int k = A.qk ? A.qk[qid] : A.k;
    const int pad = KC - k;
    const float r2 = A.r2s ? A.r2s[qid] : A.r2;
    const uint64_t empty = r2 > 0.0f ? make_key(r2, 0) : 0;
#pragma unroll
    for (int j = 0; j < KC; ++j) h[j] = j < pad ? 0 : empty;
    int2* my = stk + threadIdx.x;
    int sp = 0;
    int cur = query_root(A, qid);
    NodeRec r{};
    float bb[2 * D];
    if (cur >= 0) {
        r = nodes[cur];
        load_box<D>(bbox + (int64_t)cur * (2 * D), bb);
    }
    int lstart = 0, lcnt = 0;
    // the next pending far child whose bound does not exceed thr, or -1
    auto pop = [&](float thr) {
        while (sp > 0) {
            --sp;
            const int2 e = my[sp * kBlock];
            if (__int_as_float(e.y) <= thr) return e.x;
        }
        return -1;
    };
    while (true) {
        if constexpr (STATS) w_round += first_active_lane();
        while (true) {
            const bool walking = cur != -1 && lcnt == 0;
            const unsigned long long wb = __ballot(walking);
            if (wb == 0) break;
            const int held = __popcll(__ballot(lcnt > 0));
            if (held * 64 >= batch * (held + __popcll(wb))) break;
            if (walking) {
                if constexpr (STATS) {
                    ++n_step;
                    w_step += first_active_lane();
                }
                const float thr = key_dist(h[KC - 1]);
                int next;
                if (cur == kPopAfterScan) {
                    next = pop(thr);
                } else {
                    if constexpr (STATS) ++n_enter;
                    const float b = box_bound<D>(q, bb);
                    if (b > thr) {  // no point of this node can enter H
                        next = pop(thr);
                    } else if (r.dim < 0) {  // a bucket: scan it, then pop
                        lstart = r.a;
                        lcnt = -r.dim;
                        next = kPopAfterScan;
                    } else {
                        const float qd = select_dim<D>(q, r.dim);
                        const bool left_near = qd < r.split;
                        const float o = left_near ? r.split - qd : qd - r.split;
                        if (sp < sdepth) {  // always: a path holds at most depth pending entries
                            my[sp * kBlock] =
                                make_int2(left_near ? r.a + 1 : r.a, __float_as_int(o * o));
                            ++sp;
                        }
                        next = left_near ? r.a : r.a + 1;  // near child first
                    }
                }
                cur = next;
                if (cur >= 0) {
                    r = nodes[cur];
                    load_box<D>(bbox + (int64_t)cur * (2 * D), bb);
                }
            }
        }
        if (__ballot(lcnt > 0) == 0) break;  // no lane walks and none holds a bucket
        if constexpr (STATS) {
            n_leaf += lcnt > 0;
            n_pts += lcnt;
        }
        constexpr int B = RB;
        static_assert(B <= kRowPad, "row batches must fit in the padding rows");
        const float* row0 = pts + (int64_t)lstart * (D + 1);
        if (__ballot(lcnt > 0 && h[KC - 1] == empty) != 0) {
            for (int j0 = 0; j0 < lcnt; j0 += B) {
                if constexpr (STATS) w_rows += first_active_lane();
                float x[B][D + 1];
#pragma unroll
                for (int b = 0; b < B; ++b) load_row<D>(row0 + (j0 + b) * (D + 1), x[b]);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int id = __float_as_int(x[b][D]);
                    const uint64_t key = make_key(distance<D>(q, x[b]), id);
                    if (j0 + b < lcnt && key < h[KC - 1] && id != self) {
                        if constexpr (STATS) {
                            ++n_ins;
                            w_ins += first_active_lane();
                        }
                        heap_insert<KC>(h, key);
                    }
                }
            }
        } else {
            for (int j0 = 0; j0 < lcnt; j0 += B) {
                if constexpr (STATS) w_rows += first_active_lane();
                float x[B][D + 1];
#pragma unroll
                for (int b = 0; b < B; ++b) load_row<D>(row0 + (j0 + b) * (D + 1), x[b]);
                uint64_t keys[B];
                unsigned cand = 0;
                const uint64_t top = h[KC - 1];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int id = __float_as_int(x[b][D]);
                    keys[b] = make_key(distance<D>(q, x[b]), id);
                    if (j0 + b < lcnt && keys[b] < top && id != self) cand |= 1u << b;
                }
                while (cand) {
                    const int j = __builtin_ctz(cand);
                    cand &= cand - 1;
                    uint64_t key = keys[0];
#pragma unroll
                    for (int b = 1; b < B; ++b) key = j == b ? keys[b] : key;
                    if (key < h[KC - 1]) {
                        if constexpr (STATS) {
                            ++n_ins;
                            w_ins += first_active_lane();
                        }
                        heap_insert<KC>(h, key);
                    }
                }
            }
        }
        lcnt = 0;
    }
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        if (j >= pad) {
            const int64_t o = (A.qout ? A.qout[qid] : qid * k) + (j - pad);
            const bool none = h[j] == empty;
            A.out_idx[o] = none ? -1 : (int)(uint32_t)h[j];
            A.out_d2[o] = none ? INFINITY : key_dist(h[j]);
        }
    }
    }  // slot < m
    if constexpr (STATS) {
        unsigned long long c[9] = {n_enter, n_leaf, n_pts, n_step, n_ins,
                                   w_step, w_rows, w_round, w_ins};
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            for (int o = 32; o > 0; o >>= 1) c[j] += __shfl_xor(c[j], o);
            if ((threadIdx.x & 63) == 0) atomicAdd(&A.stats[j], c[j]);
        }
    }
}

// One wavefront per query: Algorithm 1's depth-first search with the
// explicit stack run by the whole wavefront, for deep searches (high
// dimensions, large k) where a lane-per-query walk leaves one lane to scan
// thousands of buckets alone.  The control flow is uniform: the stack of
// pending far children is held across the lanes (entry i in lane i, at most
// 64 entries), a bucket's rows are scanned one row per lane, and the heap is
// a sorted list of 64-bit (distance, index) keys, entry j in lane j < k; the
// rows of a bucket that beat the k-th key are inserted one after the other.
// Pruning and the result are those of k_traverse_stack.
__device__ inline uint64_t readlane_u64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_traverse_wave(TravArgs A)
{
    const NodeRec* __restrict__ nodes = A.nodes;
    const float* __restrict__ bbox = A.bbox;
    const float* __restrict__ pts = A.pts;
    const int lane = threadIdx.x & 63;
    const int64_t slot =
        (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (slot >= A.m) return;  // the whole wavefront
    const int64_t qid = A.order ? A.order[slot] : slot;
    float q[D];
#pragma unroll
    for (int t = 0; t < D; ++t) q[t] = A.queries[qid * D + t];
    const int32_t self = A.self_ids ? A.self_ids[qid] : -1;
    const int k = __builtin_amdgcn_readfirstlane(A.qk ? A.qk[qid] : A.k);
    const float r2 = A.r2s ? A.r2s[qid] : A.r2;
    const uint64_t empty = r2 > 0.0f ? make_key(r2, 0) : 0;
    uint64_t h = empty;  // lane j < k: the (j + 1)-th smallest key so far
    int s_node = 0;      // pending far child of stack entry `lane`
    float s_bound = 0.0f;
    int sp = 0;
    int cur = 0;
    if (A.root) {  // one lane validates (and counts) the tree id for the wavefront
        int r0 = 0;
        if (lane == 0) r0 = query_root(A, qid);
        cur = __builtin_amdgcn_readfirstlane(r0);
    }
    // record and box of the stack's top entry, loaded while a bucket is
    // scanned: the node the next pop most likely returns
    int pf = -1;
    NodeRec pr{};
    float pbb[2 * D];
    while (true) {
        uint64_t top = readlane_u64(h, k - 1);
        const float thr = key_dist(top);
        if (cur < 0) {  // the next pending far child whose bound does not exceed thr
            while (sp > 0) {
                --sp;
                const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s_bound), sp));
                if (b <= thr) {
                    cur = __builtin_amdgcn_readlane(s_node, sp);
                    break;
                }
            }
            if (cur < 0) break;
        }
        NodeRec r;
        float bb[2 * D];
        if (cur == pf) {
            r = pr;
#pragma unroll
            for (int t = 0; t < 2 * D; ++t) bb[t] = pbb[t];
        } else {
            r = nodes[cur];
            load_box<D>(bbox + (int64_t)cur * (2 * D), bb);
        }
        pf = -1;
        if (box_bound<D>(q, bb) > thr) {  // no point of this node can enter H
            cur = -1;
            continue;
        }
        if (r.dim >= 0) {
            const float qd = select_dim<D>(q, r.dim);
            const bool left_near = qd < r.split;
            const float o = left_near ? r.split - qd : qd - r.split;
            if (sp < kWave) {  // always: a path holds at most depth pending entries
                if (lane == sp) {
                    s_node = left_near ? r.a + 1 : r.a;
                    s_bound = o * o;
                }
                ++sp;
            }
            cur = left_near ? r.a : r.a + 1;  // near child first
            continue;
        }
        const int cnt = -r.dim;
        if (sp > 0) {
            pf = __builtin_amdgcn_readlane(s_node, sp - 1);
            pr = nodes[pf];
            load_box<D>(bbox + (int64_t)pf * (2 * D), pbb);
        }
        for (int j0 = 0; j0 < cnt; j0 += kWave) {
            const int j = j0 + lane;
            uint64_t key = ~0ull;
            bool cand = false;
            if (j < cnt) {
                float x[D + 1];
                load_row<D>(pts + (int64_t)(r.a + j) * (D + 1), x);
                const int id = __float_as_int(x[D]);
                key = make_key(distance<D>(q, x), id);
                cand = key < top && id != self;
            }
            uint64_t cm = __ballot(cand);
            while (cm) {
                const int src = __builtin_ctzll(cm);
                cm &= cm - 1;
                const uint64_t kk = readlane_u64(key, src);
                if (kk < top) {  // insert into the sorted list, dropping entry k - 1
                    const uint32_t plo = (uint32_t)__shfl_up((int)(uint32_t)h, 1);
                    const uint32_t phi = (uint32_t)__shfl_up((int)(uint32_t)(h >> 32), 1);
                    const uint64_t prev = ((uint64_t)phi << 32) | plo;
                    if (lane < k && kk < h) h = (lane > 0 && kk < prev) ? prev : kk;
                    top = readlane_u64(h, k - 1);
                }
            }
        }
        cur = -1;
    }
    if (lane < k) {
        const int64_t o = (A.qout ? A.qout[qid] : qid * k) + lane;
        const bool none = h == empty;
        A.out_idx[o] = none ? -1 : (int)(uint32_t)h;
        A.out_d2[o] = none ? INFINITY : key_dist(h);
    }
}

using WaveFn = void (*)(TravArgs);

// Home leaf of every query: descend with the near-child rule (x < split
// left).  Queries are grouped by key = (first packed position of the home
// leaf) >> shift: buckets are contiguous in packed order, so key order is the
// tree's spatial order.  Each lane descends kLocQ queries at once (blocks of
// kBlock * kLocQ consecutive queries, lane t taking t, t + kBlock, ...), so
// that kLocQ independent node loads are in flight per step.
constexpr int kLocQ = 4;

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

__global__ __launch_bounds__(kBlock) void k_zero(uint32_t* __restrict__ a, int64_t len)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < len) a[i] = 0u;
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

using TraverseFn = void (*)(TravArgs);
using LocateFn = void (*)(const NodeRec*, const float*, const int32_t*, int32_t, int64_t, int,
                          int32_t*, uint32_t*);

template <int D, bool STATS>
TraverseFn pick_traverse(int k)
{
    constexpr int RB = D <= 10 ? 8 : 4;  // bucket rows per batch
    if (k <= 4) return k_traverse<D, 4, STATS, RB>;
    if (k <= 8) return k_traverse<D, 8, STATS, RB>;
    if (k <= 16) return k_traverse<D, 16, STATS, RB>;
    if (k <= 32) return k_traverse<D, 32, STATS, RB>;
    return k_traverse<D, 64, STATS, RB>;
}

using StackFn = void (*)(TravArgs, int);

template <int D, bool STATS>
StackFn pick_stack(int k)
{
    constexpr int RB = D <= 10 ? 8 : 4;
    if (k <= 4) return k_traverse_stack<D, 4, STATS, RB>;
    if (k <= 8) return k_traverse_stack<D, 8, STATS, RB>;
    if (k <= 16) return k_traverse_stack<D, 16, STATS, RB>;
    if (k <= 32) return k_traverse_stack<D, 32, STATS, RB>;
    return k_traverse_stack<D, 64, STATS, RB>;
}

StackFn stack_for(int d, int k, bool stats)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return stats ? pick_stack<DD, true>(k) : pick_stack<DD, false>(k);
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4)
        KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
        KNN_DIM_CASE(9) KNN_DIM_CASE(10) KNN_DIM_CASE(11) KNN_DIM_CASE(12)
        KNN_DIM_CASE(13) KNN_DIM_CASE(14) KNN_DIM_CASE(15) KNN_DIM_CASE(16)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
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
    // one wavefront per query (the tree's depth bounds the lanes' stack):
    // asked for, or by default for batches too small to fill the device with
    // one lane per query; it runs in input order (grouping by home leaf costs
    // more than the coherence it buys a wavefront that walks one query)
    const bool wave_ok = t->depth + 1 <= kWave && qs.stats == nullptr;
    const bool use_wave =
        wave_ok && (qs.traversal == 3 || (qs.traversal == 0 && m <= kWaveQueriesMax));
    const bool grouped = qs.order != 1 && !use_wave;
    // key range: packed positions >> shift, at most 2^22 buckets
    int shift = 0;
    while ((t->n >> shift) > (int64_t(1) << 22)) ++shift;
    const int64_t N = grouped ? (t->n >> shift) + 1 : 0;
    const int64_t nsb = (N + kScanChunk - 1) / kScanChunk;
    const int64_t mg = grouped ? m : 0;
    // workspace: cnt[N], block sums[nsb], home[m], order[m], shome[m]
    const size_t bytes = sizeof(uint32_t) * (size_t)(N + nsb) + sizeof(int32_t) * 3 * (size_t)mg;
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
        KNN_HIP(hipMallocAsync(&ws.p, bytes, st));
        base = ws.p;
    }
    uint32_t* cnt = static_cast<uint32_t*>(base);
    uint32_t* bsum = cnt + N;
    int32_t* home = reinterpret_cast<int32_t*>(bsum + nsb);
    int32_t* ord = home + mg;
    int32_t* shome = ord + mg;
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
        k_scan_add<<<(unsigned)((N + kBlock - 1) / kBlock), kBlock, 0, st>>>(cnt, N, bsum);
        k_group<<<grid, kBlock, 0, st>>>(t->nodes, home, m, shift, cnt, ord, shome);
        KNN_HIP(hipGetLastError());
    }
    prof_mark(st, 7);
    TravArgs A{};
    A.nodes = t->nodes;
    A.bbox = t->bbox;
    A.pts = t->pts;
    A.queries = qs.queries;
    A.order = grouped ? ord : nullptr;
    A.home = grouped ? shome : nullptr;
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
                           (qs.traversal == 2 || (qs.traversal == 0 && d >= kStackMinDim));
    if (use_wave) {
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
