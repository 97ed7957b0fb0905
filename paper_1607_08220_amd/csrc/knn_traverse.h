// Traversal kernels of the batched k-NN query (Algorithm 1, Sections
// III-B/III-C of arXiv 1607.08220), shared by the translation units that
// instantiate them: knn_trav_lane*.hip (one lane per query, stack-free walk),
// knn_trav_stack*.hip (one lane per query, explicit stack in LDS) and
// knn_query.hip (one wavefront per query, and the host side).
//
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
#pragma once

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
// default from kStackMinDim dimensions: batches above kWaveQueriesMaxHigh and
// up to kTeamQueriesMax queries take a team of kTeamDefault lanes per query
constexpr int64_t kWaveQueriesMaxHigh = 4096;
constexpr int64_t kTeamQueriesMax = 32768;
constexpr int kTeamDefault = 32;

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
    const int2* slots;      // grouped order: slot -> (query, its home leaf); NULL: input order
    bool start_home;        // the lane-per-query walk starts at the home leaf (else the root)
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
    const int2* __restrict__ slots = A.slots;
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
    const int2 sl = slots ? slots[slot] : make_int2(0, 0);
    const int64_t qid = slots ? (int64_t)sl.x : slot;
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
    int cur = root < 0 ? -1 : (slots && A.start_home ? sl.y : root);
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
    const int64_t qid = A.slots ? (int64_t)A.slots[slot].x : slot;
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

// The k nearest neighbours of one query, computed by the whole (active,
// uniform) wavefront: q is the query, self the index it excludes (-1: none),
// r2 the squared radius, root the node to start at (-1: none, padding rows),
// k the neighbour count; lane j < k writes entry j to out_idx / out_d2.
template <int D>
__device__ inline void wave_answer(const NodeRec* __restrict__ nodes,
                                   const float* __restrict__ bbox, const float* __restrict__ pts,
                                   const float (&q)[D], int32_t self, int k, float r2, int root,
                                   int32_t* __restrict__ out_idx, float* __restrict__ out_d2)
{
    const int lane = threadIdx.x & 63;
    const uint64_t empty = r2 > 0.0f ? make_key(r2, 0) : 0;
    uint64_t h = empty;  // lane j < k: the (j + 1)-th smallest key so far
    int s_node = 0;      // pending far child of stack entry `lane`
    float s_bound = 0.0f;
    int sp = 0;
    int cur = root;
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
        const bool none = h == empty;
        out_idx[lane] = none ? -1 : (int)(uint32_t)h;
        out_d2[lane] = none ? INFINITY : key_dist(h);
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_traverse_wave(TravArgs A)
{
    const int lane = threadIdx.x & 63;
    const int64_t slot =
        (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (slot >= A.m) return;  // the whole wavefront
    const int64_t qid = A.slots ? (int64_t)A.slots[slot].x : slot;
    float q[D];
#pragma unroll
    for (int t = 0; t < D; ++t) q[t] = A.queries[qid * D + t];
    const int32_t self = A.self_ids ? A.self_ids[qid] : -1;
    const int k = __builtin_amdgcn_readfirstlane(A.qk ? A.qk[qid] : A.k);
    const float r2 = A.r2s ? A.r2s[qid] : A.r2;
    int cur = 0;
    if (A.root) {  // one lane validates (and counts) the tree id for the wavefront
        int r0 = 0;
        if (lane == 0) r0 = query_root(A, qid);
        cur = __builtin_amdgcn_readfirstlane(r0);
    }
    const int64_t o = A.qout ? A.qout[qid] : qid * k;
    wave_answer<D>(A.nodes, A.bbox, A.pts, q, self, k, r2, cur, A.out_idx + o, A.out_d2 + o);
}

// A team of T lanes (T divides 64) per query: the one-wavefront-per-query
// search above with the wavefront split into 64 / T independent teams, for
// batches large enough to fill the device with teams.  Team lane i holds
// stack entry i and, for i < k, heap entry i; a bucket is scanned T rows at
// a time; every exchange stays inside the team (shuffles of width T, the
// team's bits of a ballot).  Needs k <= T and depth + 1 <= T.  Control flow
// is uniform within a team only.
__device__ inline uint64_t team_read_u64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <int D, int T>
__device__ inline void team_answer(const NodeRec* __restrict__ nodes,
                                   const float* __restrict__ bbox, const float* __restrict__ pts,
                                   const float (&q)[D], int32_t self, int k, float r2, int root,
                                   int32_t* __restrict__ out_idx, float* __restrict__ out_d2)
{
    static_assert(T >= 2 && T <= kWave && (kWave % T) == 0, "a team divides the wavefront");
    const int lane = threadIdx.x & 63;
    const int tl = lane & (T - 1);  // lane within the team
    const int tb = lane - tl;       // the team's first lane
    constexpr uint64_t kTeamBits = T == 64 ? ~0ull : ((1ull << T) - 1);
    const uint64_t empty = r2 > 0.0f ? make_key(r2, 0) : 0;
    uint64_t h = empty;  // team lane j < k: the (j + 1)-th smallest key so far
    int s_node = 0;      // pending far child of stack entry tl
    float s_bound = 0.0f;
    int sp = 0;
    int cur = root;
    int pf = -1;  // the stack top's node, loaded while a bucket is scanned
    NodeRec pr{};
    float pbb[2 * D];
    while (true) {
        uint64_t top = team_read_u64(h, tb + k - 1);
        const float thr = key_dist(top);
        if (cur < 0) {  // the next pending far child whose bound does not exceed thr
            while (sp > 0) {
                --sp;
                const float b = __shfl(s_bound, tb + sp);
                if (b <= thr) {
                    cur = __shfl(s_node, tb + sp);
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
            if (sp < T) {  // always: a path holds at most depth pending entries
                if (tl == sp) {
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
            pf = __shfl(s_node, tb + sp - 1);
            pr = nodes[pf];
            load_box<D>(bbox + (int64_t)pf * (2 * D), pbb);
        }
        for (int j0 = 0; j0 < cnt; j0 += T) {
            const int j = j0 + tl;
            uint64_t key = ~0ull;
            bool cand = false;
            if (j < cnt) {
                float x[D + 1];
                load_row<D>(pts + (int64_t)(r.a + j) * (D + 1), x);
                const int id = __float_as_int(x[D]);
                key = make_key(distance<D>(q, x), id);
                cand = key < top && id != self;
            }
            uint64_t cm = (__ballot(cand) >> tb) & kTeamBits;
            while (cm) {
                const int src = __builtin_ctzll(cm);
                cm &= cm - 1;
                const uint64_t kk = team_read_u64(key, tb + src);
                if (kk < top) {  // insert into the sorted list, dropping entry k - 1
                    const uint32_t plo = (uint32_t)__shfl_up((int)(uint32_t)h, 1, T);
                    const uint32_t phi = (uint32_t)__shfl_up((int)(uint32_t)(h >> 32), 1, T);
                    const uint64_t prev = ((uint64_t)phi << 32) | plo;
                    if (tl < k && kk < h) h = (tl > 0 && kk < prev) ? prev : kk;
                    top = team_read_u64(h, tb + k - 1);
                }
            }
        }
        cur = -1;
    }
    if (tl < k) {
        const bool none = h == empty;
        out_idx[tl] = none ? -1 : (int)(uint32_t)h;
        out_d2[tl] = none ? INFINITY : key_dist(h);
    }
}

template <int D, int T>
__global__ __launch_bounds__(kBlock) void k_traverse_team(TravArgs A)
{
    constexpr int kQpw = kWave / T;  // queries per wavefront
    const int lane = threadIdx.x & 63;
    const int tb = lane & ~(T - 1);
    const int64_t slot = ((int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)) * kQpw + lane / T;
    if (slot >= A.m) return;  // the whole team
    const int64_t qid = A.slots ? (int64_t)A.slots[slot].x : slot;
    float q[D];
#pragma unroll
    for (int t = 0; t < D; ++t) q[t] = A.queries[qid * D + t];
    const int32_t self = A.self_ids ? A.self_ids[qid] : -1;
    const int k = A.qk ? A.qk[qid] : A.k;
    const float r2 = A.r2s ? A.r2s[qid] : A.r2;
    int cur = 0;
    if (A.root) {  // the team's first lane validates (and counts) the tree id
        int r0 = 0;
        if (lane == tb) r0 = query_root(A, qid);
        cur = __shfl(r0, tb);
    }
    const int64_t o = A.qout ? A.qout[qid] : qid * k;
    team_answer<D, T>(A.nodes, A.bbox, A.pts, q, self, k, r2, cur, A.out_idx + o, A.out_d2 + o);
}

}  // namespace

using TraverseFn = void (*)(TravArgs);
using StackFn = void (*)(TravArgs, int);

// The lane-per-query kernel for dimension d and heap capacity >= k (with or
// without visit counters): knn_trav_lane1.hip (d <= 8), knn_trav_lane2.hip.
TraverseFn traverse_for_low(int d, int k, bool stats);
TraverseFn traverse_for_high(int d, int k, bool stats);
// The explicit-stack kernel likewise: knn_trav_stack1.hip, knn_trav_stack2.hip.
StackFn stack_for_low(int d, int k, bool stats);
StackFn stack_for_high(int d, int k, bool stats);
// The team form for dimension d and team size t in {8, 16, 32}:
// knn_trav_team.hip.
TraverseFn team_for(int d, int t);

}  // namespace knn
