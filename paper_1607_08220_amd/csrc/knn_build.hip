// kd-tree construction on gfx950 (Section III-A of arXiv 1607.08220).
//
// The paper builds the local tree breadth-first with all threads on the top
// levels (III-A ii), then lets each thread finish a subtree depth-first
// (III-A iii), then packs buckets (III-A iv).  Here:
//   * ingest:    caller AoS [n,d] -> SoA columns + index column
//   * level pass (nodes above `W` points), one node list per level:
//       k_sample   one wavefront per node: sample of min(1024, cnt) points
//                  (read whole from the slot the previous partition filled,
//                  for nodes of at least 4096 points), FP64 variance per dim,
//                  split dim = argmax, the sample of that dim sorted in
//                  registers; keeps the ranks around the middle that the
//                  histogram resolves
//       k_hist     counts below that window of ranks and the bins inside it
//                  (per-wavefront LDS queue, LDS binary search), per node and
//                  as a prefix row per partition block
//       k_choose   C_j over the window, j* = argmin |2 C_j - cnt| once the
//                  window is shown to hold it, else the node's full histogram
//                  (k_choose_wave: the same with one wavefront per node); then
//                  each partition block's left count (a read of its prefix
//                  row) and their exclusive scan over the node
//       k_plan_*   children ids, next level's node list and block tables,
//                  sample slots, subtree entries: prefix sums on the device
//       k_scatter  stable partition of coordinates + index into the other
//                  ping-pong buffer (ballot + mbcnt ranks, LDS staging); also
//                  copies the large children's samples into their slots
//   * k_finish:  one wavefront per node of at most W points builds its whole
//                subtree in LDS (every point is a sample there, so the split
//                is the exact value the histogram rule selects), computes the
//                tight boxes and writes the packed bucket rows
//   * k_compact: gives every subtree node its final id; k_bbox_up fills the
//                boxes of the level-pass nodes bottom-up.
// Node ids are deterministic: the roots first (tree t of a forest is node t),
// then level-pass nodes in breadth-first order, then each subtree's nodes in
// the order the subtree list is kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <vector>

#include "knn_internal.h"

namespace knn {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;       // 4
constexpr int kItems = 16;                           // elements per lane per block pass
constexpr int kChunk = kBlock * kItems;              // 4096 elements per block
constexpr int kBins = kSampleMax + 1;                // histogram bins per node (full)
// The level histogram only resolves the sample ranks jl..jh around the middle
// (jl = s/2 - kWinHalf, jh = s/2 + kWinHalf, clamped): a node's row holds
// [#{x < s_jl}, the bins jl+1..jh] (entries 0 .. jh - jl).
constexpr int kWinHalf = 128;
constexpr int kWinRow = 2 * kWinHalf + 2;
constexpr int kWinStride = 2 * kWinHalf + 8;  // sorted sample values s_jl..s_jh per node
// The histogram pass gives each block 8 times more points: every block adds
// its LDS histogram into the node's global one, so fewer blocks mean fewer
// global atomics on the same counters.
constexpr int kHistChunk = 8 * kChunk;
constexpr int kSubs = kHistChunk / kChunk;  // partition blocks per histogram block
// The histogram pass also leaves, for every partition block of kChunk points,
// the inclusive prefix of the block's own window row: entry m is the number
// of the block's points below s_(jl + m), so once the split s_j is chosen the
// block's left count is one read at m = j - jl (counts <= kChunk fit 16 bits).
constexpr int kCrowStride = kWinRow;
static_assert(kChunk <= 65535, "per-block prefix counts are stored in 16 bits");
constexpr int kStack = 32;                           // subtree DFS stack (entries)
// Children of at least this many points that need another level pass get
// their sample written by the partition that creates them (1024 values per
// dimension, in a slot of the pre-gathered sample buffer), so the next
// level's sampler reads it whole instead of gathering strided points: from
// 4096 points on the strided gather fetches more lines than the slot costs
// to write and read.
constexpr int kPreSampleMin = 4 * kSampleMax;

// A subtree handed to the finish kernel: points [start, start + count) of
// ping-pong buffer `buf`, node id, parent id, depth of its root; leaf_only
// marks a bucket that is not split further (at most `leaf` points, or all
// points identical).
struct SubEntry {
    int32_t start, count, node_id, parent;
    int32_t buf, leaf_only, depth0, pad;
};

// One level of the level passes, all in device memory: the node list
// (start, count, id, parent, depth, pre-gathered sample slot or -1), each
// node's blocks of kChunk points (blk0, nblk) and the block tables (bnode,
// bbeg for kChunk blocks; hnode, hbeg for kHistChunk blocks).
// cnt = {nodes, blocks, histogram blocks}.
// Kernels are launched with grids sized for the largest possible level and
// return at once past these counts, so no level needs a host round trip.
struct Level {
    int32_t* start;
    int32_t* count;
    int32_t* id;
    int32_t* parent;
    int32_t* depth;
    int32_t* blk0;
    int32_t* nblk;
    int32_t* bnode;
    int32_t* bbeg;
    int32_t* hnode;
    int32_t* hbeg;
    int32_t* hblk0;
    int32_t* sslot;
    int32_t* cnt;
};

// Build-wide device counters (the id and subtree counters before the
// current level are kept in G_BASE_ID / G_BASE_SUB for the plan writes).
// G_MOVED: 64-bit count of points partitioned (slots 6-7).
// G_NONFINITE: set by the ingest when an input coordinate is NaN or infinite.
// G_LEVEL_NODES: nodes of the level the latest pass wrote (its cnt[0]).
enum { G_NEXT_ID = 0, G_NSUB = 1, G_ERR = 2, G_BASE_ID = 3, G_BASE_SUB = 4, G_MOVED = 6,
       G_NONFINITE = 8, G_LEVEL_NODES = 9, G_COUNT = 10 };
// split nodes, level children, subtrees, blocks, histogram blocks, children
// with a pre-gathered sample
constexpr int kPlanVals = 6;
constexpr int kPlanStride = 8;
constexpr int kErrOverflow = -100;

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__host__ __device__ inline int64_t sample_pos(int64_t j, int64_t c, int64_t s)
{
    return ((2 * j + 1) * c) / (2 * s);
}

__device__ inline float wave_min(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}


// ---------------------------------------------------------------------------
// B0: ingest
// ---------------------------------------------------------------------------
// Also flags (g[G_NONFINITE]) an input coordinate that is NaN or infinite:
// the build requires finite points.
__global__ void k_ingest(const float* __restrict__ aos, int64_t n, int d,
                         float* __restrict__ cols, int32_t* __restrict__ idx,
                         int32_t* __restrict__ g)
{
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int t = 0; t < d; ++t) {
            const float v = aos[i * d + t];
            bad = bad || !__builtin_isfinite(v);
            cols[(int64_t)t * n + i] = v;
        }
        idx[i] = (int32_t)i;
    }
    if (__ballot(bad) != 0 && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&g[G_NONFINITE], 1);
}

// ---------------------------------------------------------------------------
// B1-B3: sample, split dimension, sorted sample (one block per node)
// ---------------------------------------------------------------------------
__device__ inline void sample_window(int s, int* jl, int* jh)
{
    *jl = s / 2 - kWinHalf > 0 ? s / 2 - kWinHalf : 0;
    *jh = s / 2 + kWinHalf < s - 1 ? s / 2 + kWinHalf : s - 1;
}

// Sample position of rank j (s = kSampleMax is a power of two: a shift).
__device__ inline int64_t sample_pos_fast(int64_t j, int64_t c, int s)
{
    return s == kSampleMax ? ((2 * j + 1) * c) >> 11 : sample_pos(j, c, s);
}
static_assert(2 * kSampleMax == 2048, "sample_pos_fast divides by 2 * kSampleMax with a shift");

// Pairwise FP64 sum over a[0..1023] (zero padded past the sample size):
// a[i] += a[i + w] for w = 512, 256, .., 1, the total in a[0].  Zero padding
// leaves the sum equal to the same tree over the next power of two above the
// sample size.  One wavefront: lane L holds a[L + 64 r], r = 0..15, so the
// strides 512..64 stay inside the lane and 32..1 cross lanes.  The result is
// returned to every lane.
__device__ inline double wave_psum(double (&v)[16])
{
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = v[r] + v[r + 8];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = v[r] + v[r + 4];
#pragma unroll
    for (int r = 0; r < 2; ++r) v[r] = v[r] + v[r + 2];
    double x = v[0] + v[1];
    for (int w = 32; w >= 1; w >>= 1) x = x + __shfl_down(x, w);
    return __shfl(x, 0);
}

// Bitonic sort of 1024 floats held by one wavefront, element 16 L + r in
// register r of lane L: strides below 16 stay in the lane, the others pair
// lane L with lane L ^ (stride / 16).
__device__ inline void wave_sort1024(float (&u)[16])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= 1024; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 16) {
                const int lm = j >> 4;
                const bool lower = (lane & lm) == 0;
                const bool asc = k >= 16 ? ((16 * lane) & k) == 0 : true;
                const bool keep_min = lower == asc;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float p = __shfl_xor(u[r], lm);
                    u[r] = keep_min ? fminf(u[r], p) : fmaxf(u[r], p);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if ((r & j) == 0) {
                        const bool asc = k >= 16 ? ((16 * lane) & k) == 0 : (r & k) == 0;
                        const float x = u[r], y = u[r | j];
                        const float lo = fminf(x, y), hi = fmaxf(x, y);
                        u[r] = asc ? lo : hi;
                        u[r | j] = asc ? hi : lo;
                    }
                }
            }
        }
    }
}

// B1-B3: one wavefront per node (kWavesPerBlock nodes per block).  Sample
// s = min(count, 1024) points at the systematic positions, pick the
// dimension of largest sample variance (FP64, fixed pairwise order), sort
// the sample along it (kept in registers from the variance pass, moved to
// the sort's layout through LDS) and keep the values of ranks jl..jh; clear
// the node's histogram row.  Bounded to 128 registers: four wavefronts per
// SIMD, without spills.
__global__ __launch_bounds__(kBlock, 4) void k_sample(Level L, const float* __restrict__ cols,
                                                   const float* __restrict__ psamp, int64_t n,
                                                   int d, float* __restrict__ samples,
                                                   int32_t* __restrict__ out_dim,
                                                   uint32_t* __restrict__ hist)
{
    __shared__ float tr[kWavesPerBlock][kSampleMax];  // the best column's sample, transposed
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // wavefront-uniform: node data loads through the scalar unit
    const int node = blockIdx.x * kWavesPerBlock + w;
    if (node >= L.cnt[0]) return;
    const int64_t start = L.start[node], c = L.count[node];
    const int sl = L.sslot[node];  // >= 0: the partition wrote this node's sample (s = 1024)
    for (int i = lane; i < kWinRow; i += kWave) hist[(int64_t)node * kWinRow + i] = 0u;
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    double bestV = -1.0;
    int best = 0;
    float* t = tr[w];  // the sample of the best dimension so far, element j at t[j]
    for (int dd = 0; dd < d; ++dd) {
        const float* col = cols + (int64_t)dd * n + start;
        const float* pre = psamp + ((int64_t)(sl >= 0 ? sl : 0) * d + dd) * kSampleMax;
        double v[16], q[16];
        float f[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int j = lane + 64 * r;
            f[r] = sl >= 0 ? pre[j] : col[sample_pos_fast(j < s ? j : s - 1, c, s)];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = lane + 64 * r < s ? (double)f[r] : 0.0;
        const double S = wave_psum(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const double w = (double)s * (double)f[r] - S;
            q[r] = lane + 64 * r < s ? w * w : 0.0;
        }
        const double V = wave_psum(q);
        if (V > bestV) {
            bestV = V;
            best = dd;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = lane + 64 * r;
                t[j] = j < s ? f[r] : INFINITY;
            }
        }
    }
    if (!(bestV > 0.0)) {  // sample constant in every dimension
        if (lane == 0) out_dim[node] = -1;
        return;
    }
    // element j to lane j / 16, register j % 16: the sort's layout
    wave_sync();
    float u[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) u[r] = t[16 * lane + r];
    wave_sort1024(u);
    int jl, jh;
    sample_window(s, &jl, &jh);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int j = 16 * lane + r;
        if (j >= jl && j <= jh) samples[(int64_t)node * kWinStride + (j - jl)] = u[r];
    }
    if (lane == 0) out_dim[node] = best;
}

// B1-B3 for levels of few nodes: the same computation as k_sample with a
// workgroup of kSampleMax threads per node (thread t holds sample element t),
// so the few nodes of the top levels are not each left to one wavefront.
// The FP64 sums run the same pairwise tree (element t += element t + w for
// w = 512 .. 1) and the sort the same bitonic network, in LDS.
__global__ __launch_bounds__(kSampleMax) void k_sample_block(Level L,
                                                            const float* __restrict__ cols,
                                                            const float* __restrict__ psamp,
                                                            int64_t n, int d,
                                                            float* __restrict__ samples,
                                                            int32_t* __restrict__ out_dim,
                                                            uint32_t* __restrict__ hist)
{
    __shared__ double acc[kSampleMax];
    __shared__ float sv[kSampleMax];
    const int node = blockIdx.x, t = threadIdx.x;
    if (node >= L.cnt[0]) return;
    const int64_t start = L.start[node], c = L.count[node];
    for (int i = t; i < kWinRow; i += kSampleMax) hist[(int64_t)node * kWinRow + i] = 0u;
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    const bool in = t < s;
    const int64_t pos = start + sample_pos_fast(in ? t : s - 1, c, s);
    const int sl = L.sslot[node];  // >= 0: the partition wrote this node's sample (s = 1024)
    float f[16];  // this element in every dimension, all loads in flight at once
#pragma unroll
    for (int dd = 0; dd < 16; ++dd)
        f[dd] = dd >= d ? 0.0f
                        : sl >= 0 ? psamp[((int64_t)sl * d + dd) * kSampleMax + t]
                                  : cols[(int64_t)dd * n + pos];
    // pairwise sum over the 1024 elements, to every thread: strides 512 .. 64
    // through LDS, 32 .. 1 by shuffles inside the first wavefront
    auto tree = [&](double v) {
        acc[t] = v;
        __syncthreads();
        for (int w = kSampleMax / 2; w >= kWave; w >>= 1) {
            if (t < w) acc[t] = acc[t] + acc[t + w];
            __syncthreads();
        }
        if (t < kWave) {
            double x = acc[t];
            for (int w = kWave / 2; w >= 1; w >>= 1) x = x + __shfl_down(x, w);
            if (t == 0) acc[0] = x;
        }
        __syncthreads();
        const double r = acc[0];
        __syncthreads();
        return r;
    };
    double bestV = -1.0;
    int best = 0;
    float fb = 0.0f;
#pragma unroll
    for (int dd = 0; dd < 16; ++dd) {
        if (dd < d) {
            const double S = tree(in ? (double)f[dd] : 0.0);
            const double wv = (double)s * (double)f[dd] - S;
            const double V = tree(in ? wv * wv : 0.0);
            if (V > bestV) {
                bestV = V;
                best = dd;
                fb = f[dd];
            }
        }
    }
    if (!(bestV > 0.0)) {  // sample constant in every dimension
        if (t == 0) out_dim[node] = -1;
        return;
    }
    // bitonic network: partners 64 or more apart through LDS, nearer ones by
    // shuffles inside the wavefront
    float e = in ? fb : INFINITY;
    for (int k = 2; k <= kSampleMax; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            float p;
            if (j >= kWave) {
                sv[t] = e;
                __syncthreads();
                p = sv[t ^ j];
                __syncthreads();
            } else {
                p = __shfl_xor(e, j);
            }
            const bool asc = (t & k) == 0, lower = (t & j) == 0;
            e = lower == asc ? fminf(e, p) : fmaxf(e, p);
        }
    }
    int jl, jh;
    sample_window(s, &jl, &jh);
    if (t >= jl && t <= jh) samples[(int64_t)node * kWinStride + (t - jl)] = e;
    if (t == 0) out_dim[node] = best;
}

// ---------------------------------------------------------------------------
// B4: histogram over the sorted sample (blocks over node chunks)
// ---------------------------------------------------------------------------
// Counts, over the node's points x, #{x < s_jl} and the bins
// b = #{j : s_j <= x} for the points in between (jl < b <= jh), which give
// C_j = #{x < s_j} exactly for every j in [jl, jh].  Points below the window
// are counted with wavefront ballots; the points inside are first queued per
// wavefront in LDS so that every lane of a binary search over the window's
// sample values has a point to place.  The search runs over the values
// s_(jl+1) .. s_(jl+255) in breadth-first (Eytzinger) order, so that step L
// reads entries 2^L .. 2^(L+1) - 1, consecutive words in distinct banks (a
// search over the sorted order reads odd multiples of its step, up to eight
// lanes per bank).  The counts are kept per partition
// block of kChunk points (the queue carries each point's block) and leave as
// the node's row and as each block's prefix row (see kCrowStride).
__global__ __launch_bounds__(kBlock) void k_hist(Level L, const int32_t* __restrict__ dimv,
                                                 const float* __restrict__ samples,
                                                 const float* __restrict__ cols, int64_t n,
                                                 uint32_t* __restrict__ hist,
                                                 uint16_t* __restrict__ crow)
{
    static_assert(2 * kWinHalf == 256, "an eight-step search over 255 window values");
    __shared__ float ev[2 * kWinHalf];  // ev[k], k = 1..255: node k of the search tree
    __shared__ uint32_t h[kSubs][kWinRow];
    __shared__ float queue[kWavesPerBlock][2 * kWave];
    __shared__ uint8_t qsub[kWavesPerBlock][2 * kWave];
    const int b = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
    if (b >= L.cnt[2]) return;
    const int node = L.hnode[b];
    const int dim = dimv[node];
    if (dim < 0) return;
    const int64_t start = L.start[node], c = L.count[node];
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    int jl, jh;
    sample_window(s, &jl, &jh);
    const int nwin = jh - jl;  // window bins jl+1 .. jh
    const int64_t beg = L.hbeg[b];
    const int64_t end = beg + kHistChunk < c ? beg + kHistChunk : c;
    // the block's chunk: len <= kHistChunk points from position beg of the node
    const float* col = cols + (int64_t)dim * n + start + beg;
    const int len = (int)(end - beg);
    constexpr int kIlp = 8;
    constexpr int kStep = kBlock * kIlp;
    // iteration it covers elements kStep * it .. kStep * it + kStep - 1 of the
    // chunk, all in partition block it / 2 of it
    static_assert(2 * kStep == kChunk, "two histogram iterations per partition block");
    const int wbeg = w * kWave * kIlp;
    float xn[kIlp];  // the next iteration's values, loaded while this one is binned
    if (wbeg < len) {  // the first ones before the window values arrive
#pragma unroll
        for (int u = 0; u < kIlp; ++u) {  // unconditional loads, clamped in range
            const int e = wbeg + u * kWave + lane;
            xn[u] = col[e < len ? e : len - 1];
        }
    }
    // node k at depth L (2^L <= k < 2^(L+1)) holds window entry
    // (2k + 1) 2^(7-L) - 256, its in-order place; past nwin the values read
    // +inf, which an in-window point (below the entry nwin) never passes
    const float* wv = samples + (int64_t)node * kWinStride;
    for (int k = t; k < 2 * kWinHalf; k += kBlock) {
        if (k == 0) continue;
        const int L = 31 - __clz(k);
        const int e = ((2 * k + 1) << (7 - L)) - 2 * kWinHalf;
        ev[k] = e <= nwin ? wv[e] : INFINITY;
    }
    const int nsub = (len + kChunk - 1) / kChunk;  // partition blocks in the chunk
    for (int i = t; i < nsub * kWinRow; i += kBlock) (&h[0][0])[i] = 0u;
    __syncthreads();
    const float lo_v = wv[0], hi_v = wv[nwin];
    int qn = 0;  // queued points of this wavefront (uniform)
    float* qw = queue[w];
    uint8_t* qs = qsub[w];
    // place the first 64 queued points: bin = jl + 1 + #{1 <= i < nwin : s_(jl+i) <= x}
    // (the search leaves node 256 + that count)
    auto drain = [&]() {
        __builtin_amdgcn_wave_barrier();
        const float x = qw[lane];
        const int sb = qs[lane];
        int kn = 1;
#pragma unroll
        for (int step = 0; step < 8; ++step) kn = 2 * kn + (ev[kn] <= x ? 1 : 0);
        atomicAdd(&h[sb][1 + kn - 2 * kWinHalf], 1u);
        const float tail = qw[kWave + lane];
        const uint8_t tsb = qs[kWave + lane];
        if (lane < qn - kWave) {
            qw[lane] = tail;
            qs[lane] = tsb;
        }
        __builtin_amdgcn_wave_barrier();
        qn -= kWave;
    };
    for (int e0 = wbeg, it = 0; e0 < len; e0 += kStep, ++it) {
        const int sub = it >> 1;
        float x[kIlp];
#pragma unroll
        for (int u = 0; u < kIlp; ++u) x[u] = xn[u];
        if (e0 + kStep < len) {
#pragma unroll
            for (int u = 0; u < kIlp; ++u) {
                const int e = e0 + kStep + u * kWave + lane;
                xn[u] = col[e < len ? e : len - 1];
            }
        }
        const int rem = len - e0;  // points left from this iteration's first
        uint32_t below = 0;  // wavefront-uniform (ballots)
#pragma unroll
        for (int u = 0; u < kIlp; ++u) {
            const bool ok = u * kWave + lane < rem;
            below += (uint32_t)__popcll(__ballot(ok && x[u] < lo_v));
            const bool in = ok && x[u] >= lo_v && x[u] < hi_v;
            const unsigned long long m = __ballot(in);
            const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
            if (in) {
                qw[qn + off] = x[u];
                qs[qn + off] = (uint8_t)sub;
            }
            qn += __popcll(m);
            if (qn >= kWave) drain();
        }
        if (lane == 0 && below) atomicAdd(&h[sub][0], below);
    }
    if (qn > 0) {  // the last partial queue: lanes past qn place nothing
        __builtin_amdgcn_wave_barrier();
        const float x = qw[lane];
        const int sb = qs[lane];
        if (lane < qn) {
            int kn = 1;
#pragma unroll
            for (int step = 0; step < 8; ++step) kn = 2 * kn + (ev[kn] <= x ? 1 : 0);
            atomicAdd(&h[sb][1 + kn - 2 * kWinHalf], 1u);
        }
    }
    __syncthreads();
    uint32_t* row = hist + (int64_t)node * kWinRow;
    for (int i = t; i <= nwin; i += kBlock) {
        uint32_t v = 0;
        for (int sb = 0; sb < nsub; ++sb) v += h[sb][i];
        if (c <= kHistChunk) row[i] = v;  // the node's only block: its row, stored whole
        else if (v) atomicAdd(&row[i], v);
    }
    __syncthreads();
    // each partition block's row becomes its inclusive prefix (a wavefront per
    // block; lane l holds the entries 5 l .. 5 l + 4)
    for (int sb = w; sb < nsub; sb += kWavesPerBlock) {
        uint32_t v[5], sum = 0;
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const int e = 5 * lane + r;
            v[r] = e <= nwin ? h[sb][e] : 0u;
            sum += v[r];
        }
        uint32_t x = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        uint32_t run = x - sum;
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const int e = 5 * lane + r;
            run += v[r];
            if (e <= nwin) h[sb][e] = run;
        }
    }
    __syncthreads();
    const int64_t gb0 = L.blk0[node] + beg / kChunk;  // the chunk's first partition block
    for (int sb = 0; sb < nsub; ++sb) {
        uint16_t* dst = crow + (gb0 + sb) * kCrowStride;
        for (int i = t; i <= nwin; i += kBlock) dst[i] = (uint16_t)h[sb][i];
    }
}

// ---------------------------------------------------------------------------
// B5: choose the split (one block per node)
// ---------------------------------------------------------------------------
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* total, uint32_t* wsum)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
        if (i < w) base += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// Thread t holds R consecutive counts v (of the entries R*t .. R*t+R-1, the
// entry e standing for sample rank j0 + e) whose inclusive prefix sums are
// C_j = #{x < s_j}.  Returns, to every thread, the smallest key
// gap * 2048 + j over the valid j (j < jend, 0 < C_j < c), gap = |2 C_j - c|:
// the rank closest to half, ties to the smaller rank; LLONG_MAX if none.
template <int R>
__device__ long long block_split_key(const uint32_t (&v)[R], int j0, int jend, int64_t c,
                                     uint32_t* wsum, long long* gbest)
{
    const int t = threadIdx.x;
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) sum += v[r];
    uint32_t tot;
    uint32_t C = block_excl_scan(sum, &tot, wsum);
    long long key = LLONG_MAX;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + R * t + r;
        C += v[r];
        if (j < jend && C > 0 && (int64_t)C < c) {
            long long gap = 2 * (long long)C - c;
            if (gap < 0) gap = -gap;
            const long long kk = gap * 2048 + j;
            if (kk < key) key = kk;
        }
    }
    gbest[t] = key;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (t < w && gbest[t + w] < gbest[t]) gbest[t] = gbest[t + w];
        __syncthreads();
    }
    key = gbest[0];
    __syncthreads();
    return key;
}

// Children of a split node that need another level pass: more than W
// points and more than the bucket size.
__host__ __device__ inline bool needs_level_pass(int c, int W, int leaf) { return c > W && c > leaf; }

// How a node's partition blocks find their left counts once the split is
// chosen: the block's prefix row at m = j - jl (split s_j inside the
// histogram window), a count of the split column below the split value, or
// all of the block (a node that stays a bucket).
enum { kLeftPrefix = 0, kLeftCount = 1, kLeftAll = 2 };

// The node's left count and plan counters: split (0/1), children needing a
// level pass, subtree entries, the children's blocks of kChunk and
// kHistChunk points, and the children that get a pre-gathered sample.
__device__ void node_plan(int node, int cnt, int nl, bool split, int W, int leaf,
                          int32_t* __restrict__ n_left, int32_t* __restrict__ planv)
{
    n_left[node] = nl;
    int v[kPlanVals] = {};
    if (split) {
        const int cc[2] = {nl, cnt - nl};
        v[0] = 1;
        for (int k = 0; k < 2; ++k) {
            if (needs_level_pass(cc[k], W, leaf)) {
                v[1] += 1;
                v[3] += (cc[k] + kChunk - 1) / kChunk;
                v[4] += (cc[k] + kHistChunk - 1) / kHistChunk;
                v[5] += cc[k] >= kPreSampleMin;
            } else {
                v[2] += 1;
            }
        }
    } else {
        v[2] = 1;
    }
    for (int k = 0; k < kPlanVals; ++k) planv[(int64_t)node * kPlanStride + k] = v[k];
}

// Wavefront w of the block (or the calling wavefront, step 1) counts, for the
// node's partition blocks i = first, first + step, ..., the points of column
// ccol below split, into blk_off[b0 + i].
__device__ void count_block_lefts(const float* __restrict__ ccol, int64_t c, float split, int b0,
                                  int nb, int first, int step, uint32_t* __restrict__ blk_off)
{
    const int lane = threadIdx.x & 63;
    for (int i = first; i < nb; i += step) {
        const int64_t e0 = (int64_t)i * kChunk;
        const int64_t e1 = e0 + kChunk < c ? e0 + kChunk : c;
        uint32_t cnt = 0;
        for (int64_t ew = e0; ew < e1; ew += kWave) {
            const int64_t e = ew + lane;
            cnt += (uint32_t)__popcll(__ballot(e < e1 && ccol[e] < split));
        }
        if (lane == 0) blk_off[b0 + i] = cnt;
    }
}

// Left count of partition block i of a node (see kLeftPrefix).
struct BlockLefts {
    const uint16_t* crow;
    const uint32_t* counted;
    int64_t c;
    int b0, m, mode;
    __device__ uint32_t operator()(int i) const
    {
        if (mode == kLeftPrefix) return crow[(int64_t)(b0 + i) * kCrowStride + m];
        if (mode == kLeftCount) return counted[b0 + i];
        const int64_t e0 = (int64_t)i * kChunk;
        return (uint32_t)(c - e0 < kChunk ? c - e0 : kChunk);
    }
};

// Exclusive scan of the node's block left counts into blk_off[b0 ..
// b0 + nb), by the whole block (16 consecutive blocks per thread and pass);
// returns the node's left count to every thread.  A thread reads only the
// entries it writes, so the counts may come from blk_off itself.
__device__ uint32_t block_lefts_scan(const BlockLefts& lefts, int nb,
                                     uint32_t* __restrict__ blk_off, uint32_t* wsum)
{
    constexpr int R = 16;
    const int t = threadIdx.x;
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kBlock * R) {
        uint32_t v[R], sum = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = base + R * t + r;
            v[r] = i < nb ? lefts(i) : 0u;
            sum += v[r];
        }
        uint32_t tot;
        uint32_t ex = carry + block_excl_scan(sum, &tot, wsum);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = base + R * t + r;
            if (i < nb) blk_off[lefts.b0 + i] = ex;
            ex += v[r];
        }
        carry += tot;
    }
    return carry;
}

// The same by one wavefront.
__device__ uint32_t wave_lefts_scan(const BlockLefts& lefts, int nb, uint32_t* __restrict__ blk_off)
{
    constexpr int R = 16;
    const int lane = threadIdx.x & 63;
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kWave * R) {
        uint32_t v[R], sum = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = base + R * lane + r;
            v[r] = i < nb ? lefts(i) : 0u;
            sum += v[r];
        }
        uint32_t x = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        const uint32_t tot = (uint32_t)__shfl((int)x, 63);
        uint32_t ex = carry + x - sum;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = base + R * lane + r;
            if (i < nb) blk_off[lefts.b0 + i] = ex;
            ex += v[r];
        }
        carry += tot;
    }
    return carry;
}

// One block per node.  From the window counts, C_j is exact for j in
// [jl, jh]; since C_j does not decrease with j, the rank closest to half lies
// in the window whenever 2 C_jl <= c <= 2 C_jh (a rank outside the window with
// the same gap has the same C_j, hence the same sample value, as jl or jh).
// Otherwise the block counts the full histogram of the node itself.  With
// the split known, the block also gives every partition block of the node its
// number of left points before it (blk_off), the node its left count and its
// plan counters.
__global__ __launch_bounds__(kBlock) void k_choose(
    Level L, int32_t* __restrict__ dimv, const float* __restrict__ samples,
    const uint32_t* __restrict__ hist, const uint16_t* __restrict__ crow,
    const float* __restrict__ cols, int64_t n, int d, int W, int leaf,
    float* __restrict__ splitv, uint32_t* __restrict__ blk_off, int32_t* __restrict__ n_left,
    int32_t* __restrict__ planv)
{
    __shared__ uint32_t wsum[kWavesPerBlock];
    __shared__ long long gbest[kBlock];
    __shared__ float fl[kBlock], fh[kBlock];
    __shared__ float sv[kSampleMax];
    __shared__ uint32_t hfull[kBins];
    const int node = blockIdx.x, t = threadIdx.x;
    if (node >= L.cnt[0]) return;
    const int64_t start = L.start[node], c = L.count[node];
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    const int dim = dimv[node];
    int mode, m = 0, cdim = dim;
    float split;
    if (dim >= 0) {
        int jl, jh;
        sample_window(s, &jl, &jh);
        const int nwin = jh - jl;
        const uint32_t* row = hist + (int64_t)node * kWinRow;
        uint32_t v[2];
        uint64_t below = row[0], inwin = 0;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = 2 * t + r;  // entry 0 is #{x < s_jl}, entry e the bin jl + e
            v[r] = e <= nwin ? row[e] : 0u;
        }
        for (int e = 1; e <= nwin; ++e) inwin += row[e];
        long long key;
        const bool in_window = 2 * (int64_t)below <= c && 2 * (int64_t)(below + inwin) >= c;
        if (in_window) {
            key = block_split_key<2>(v, jl, jh + 1, c, wsum, gbest);
        } else {
            // the middle lies outside the window: sort the whole sample again
            // and count the full histogram of the node
            const float* scol = cols + (int64_t)dim * n + start;
            int P = 1;
            while (P < s) P <<= 1;
            for (int i = t; i < P; i += kBlock) sv[i] = i < s ? scol[sample_pos(i, c, s)] : INFINITY;
            for (int i = t; i < kBins; i += kBlock) hfull[i] = 0u;
            __syncthreads();
            for (int k = 2; k <= P; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = t; i < P; i += kBlock) {
                        const int ixj = i ^ j;
                        if (ixj > i) {
                            const float x = sv[i], y = sv[ixj];
                            const bool asc = (i & k) == 0;
                            if ((x > y) == asc) {
                                sv[i] = y;
                                sv[ixj] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            const float* col = cols + (int64_t)dim * n + start;
            for (int64_t e = t; e < c; e += kBlock) {
                const float x = col[e];
                int pos = 0;  // number of sample values <= x
                for (int step = kSampleMax; step > 0; step >>= 1) {
                    const int np = pos + step;
                    if (np <= s && sv[np - 1] <= x) pos = np;
                }
                atomicAdd(&hfull[pos], 1u);
            }
            __syncthreads();
            uint32_t vf[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) vf[r] = 4 * t + r < s ? hfull[4 * t + r] : 0u;
            key = block_split_key<4>(vf, 0, s, c, wsum, gbest);
        }
        // V > 0 guarantees a valid j; the guard only keeps the index in range
        const int j = key == LLONG_MAX ? (in_window ? jl : 0) : (int)(key % 2048);
        split = in_window ? samples[(int64_t)node * kWinStride + (j - jl)] : sv[j];
        mode = in_window ? kLeftPrefix : kLeftCount;
        m = j - jl;
    } else {
        // The sample is constant in every dimension: split the dimension of
        // largest extent at its maximum, or keep a leaf if all points coincide.
        double bext = 0.0;
        int bd = -1;
        float bhi = 0.0f;
        for (int dd = 0; dd < d; ++dd) {
            const float* col = cols + (int64_t)dd * n + start;
            float lo = INFINITY, hi = -INFINITY;
            for (int64_t e = t; e < c; e += kBlock) {
                float x = col[e];
                lo = fminf(lo, x);
                hi = fmaxf(hi, x);
            }
            fl[t] = lo;
            fh[t] = hi;
            __syncthreads();
            for (int w = kBlock / 2; w >= 1; w >>= 1) {
                if (t < w) {
                    fl[t] = fminf(fl[t], fl[t + w]);
                    fh[t] = fmaxf(fh[t], fh[t + w]);
                }
                __syncthreads();
            }
            const double ext = (double)fh[0] - (double)fl[0];
            if (ext > bext) {
                bext = ext;
                bd = dd;
                bhi = fh[0];
            }
            __syncthreads();
        }
        if (t == 0) dimv[node] = bd;  // -1 keeps a leaf
        cdim = bd;
        split = bhi;
        mode = bd >= 0 ? kLeftCount : kLeftAll;
    }
    if (t == 0) splitv[node] = split;
    const int b0 = L.blk0[node], nb = L.nblk[node];
    if (mode == kLeftCount) {  // every wavefront counts some blocks; the scan reads them all
        count_block_lefts(cols + (int64_t)cdim * n + start, c, split, b0, nb, t >> 6,
                          kWavesPerBlock, blk_off);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const BlockLefts lefts{crow, blk_off, c, b0, m, mode};
    const uint32_t nl = block_lefts_scan(lefts, nb, blk_off, wsum);
    if (t == 0) node_plan(node, (int)c, (int)nl, mode != kLeftAll, W, leaf, n_left, planv);
}

// k_choose with one wavefront per node (kWavesPerBlock nodes per block), for
// levels of many small nodes; same results.  Lane L holds the window entries
// 5 L .. 5 L + 4.  The full-histogram path sorts the sample in registers and
// counts in a per-wavefront LDS histogram.
__global__ __launch_bounds__(kBlock) void k_choose_wave(
    Level L, int32_t* __restrict__ dimv, const float* __restrict__ samples,
    const uint32_t* __restrict__ hist, const uint16_t* __restrict__ crow,
    const float* __restrict__ cols, int64_t n, int d, int W, int leaf,
    float* __restrict__ splitv, uint32_t* __restrict__ blk_off, int32_t* __restrict__ n_left,
    int32_t* __restrict__ planv)
{
    __shared__ float sv_all[kWavesPerBlock][kSampleMax];
    __shared__ uint32_t hf_all[kWavesPerBlock][kBins];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int node = blockIdx.x * kWavesPerBlock + w;
    if (node >= L.cnt[0]) return;  // only wavefront-level synchronization below
    const int64_t start = L.start[node], c = L.count[node];
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    const int dim = dimv[node];
    // smallest key gap * 2048 + j over the valid j of this lane's entries
    auto wave_key = [&](const uint32_t* v, int R, int j0, int jend) -> long long {
        uint32_t sum = 0;
        for (int r = 0; r < R; ++r) sum += v[r];
        uint32_t x = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        uint32_t C = x - sum;
        long long key = LLONG_MAX;
        for (int r = 0; r < R; ++r) {
            const int j = j0 + R * lane + r;
            C += v[r];
            if (j < jend && C > 0 && (int64_t)C < c) {
                long long gap = 2 * (long long)C - c;
                if (gap < 0) gap = -gap;
                const long long kk = gap * 2048 + j;
                if (kk < key) key = kk;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const long long y = __shfl_xor(key, o);
            key = y < key ? y : key;
        }
        return key;
    };
    int mode, m = 0, cdim = dim;
    float split;
    if (dim >= 0) {
        int jl, jh;
        sample_window(s, &jl, &jh);
        const int nwin = jh - jl;
        const uint32_t* row = hist + (int64_t)node * kWinRow;
        uint32_t v[5];
        uint64_t part = 0;
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const int e = 5 * lane + r;
            v[r] = e <= nwin ? row[e] : 0u;
            if (e >= 1) part += v[r];
        }
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
        const uint64_t below = row[0];
        const bool in_window = 2 * (int64_t)below <= c && 2 * (int64_t)(below + part) >= c;
        if (in_window) {
            const long long key = wave_key(v, 5, jl, jh + 1);
            const int j = key == LLONG_MAX ? jl : (int)(key % 2048);
            split = samples[(int64_t)node * kWinStride + (j - jl)];
            mode = kLeftPrefix;
            m = j - jl;
        } else {
            float* sv = sv_all[w];
            uint32_t* hf = hf_all[w];
            const float* col = cols + (int64_t)dim * n + start;
            float u[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = 16 * lane + r;
                u[r] = j < s ? col[sample_pos(j, c, s)] : INFINITY;
            }
            wave_sort1024(u);
#pragma unroll
            for (int r = 0; r < 16; ++r) sv[16 * lane + r] = u[r];
            for (int i = lane; i < kBins; i += kWave) hf[i] = 0u;
            wave_sync();
            for (int64_t e = lane; e < c; e += kWave) {
                const float x = col[e];
                int pos = 0;  // number of sample values <= x
                for (int step = kSampleMax; step > 0; step >>= 1) {
                    const int np = pos + step;
                    if (np <= s && sv[np - 1] <= x) pos = np;
                }
                atomicAdd(&hf[pos], 1u);
            }
            wave_sync();
            uint32_t vf[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) vf[r] = 16 * lane + r < s ? hf[16 * lane + r] : 0u;
            const long long key = wave_key(vf, 16, 0, s);
            split = sv[key == LLONG_MAX ? 0 : (int)(key % 2048)];
            mode = kLeftCount;
        }
    } else {
        // the sample is constant in every dimension (see k_choose)
        double bext = 0.0;
        int bd = -1;
        float bhi = 0.0f;
        for (int dd = 0; dd < d; ++dd) {
            const float* col = cols + (int64_t)dd * n + start;
            float lo = INFINITY, hi = -INFINITY;
            for (int64_t e = lane; e < c; e += kWave) {
                const float x = col[e];
                lo = fminf(lo, x);
                hi = fmaxf(hi, x);
            }
            lo = wave_min(lo);
            hi = wave_max(hi);
            const double ext = (double)hi - (double)lo;
            if (ext > bext) {
                bext = ext;
                bd = dd;
                bhi = hi;
            }
        }
        if (lane == 0) dimv[node] = bd;
        cdim = bd;
        split = bhi;
        mode = bd >= 0 ? kLeftCount : kLeftAll;
    }
    if (lane == 0) splitv[node] = split;
    const int b0 = L.blk0[node], nb = L.nblk[node];
    if (mode == kLeftCount) {  // lane 0 writes the counts, every lane reads some
        count_block_lefts(cols + (int64_t)cdim * n + start, c, split, b0, nb, 0, 1, blk_off);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const BlockLefts lefts{crow, blk_off, c, b0, m, mode};
    const uint32_t nl = wave_lefts_scan(lefts, nb, blk_off);
    if (lane == 0) node_plan(node, (int)c, (int)nl, mode != kLeftAll, W, leaf, n_left, planv);
}

// ---------------------------------------------------------------------------
// B6: stable partition (the per-node block offsets come from k_choose)
// ---------------------------------------------------------------------------
// The block's chunk of kChunk points is reordered in LDS so that every
// column leaves as two contiguous runs (its left part, then its right part):
// element e = 256 r + thread goes to slot rank(e) of the chunk's output.
// The kLarge instance, for the levels whose children can hold kPreSampleMin
// points: a child with a pre-gathered sample slot (cslot) also gets, from
// each coordinate column, the values at its sample positions that fall in
// this chunk's run for it, and the split column is moved first, staged from
// the key loads, so the block reads it once.  The other levels (small nodes,
// many short blocks) take the plain instance, which reads the split column
// again with the others but needs 94 registers instead of 116: a wavefront
// more per SIMD, which those levels need more than the bytes.
template <bool kLarge>
__global__ __launch_bounds__(kBlock) void k_scatter(
    Level L, const int32_t* __restrict__ dimv, const float* __restrict__ splitv,
    const uint32_t* __restrict__ blk_off, const int32_t* __restrict__ n_left,
    const int32_t* __restrict__ cslot, int64_t ps_cap, const float* __restrict__ src_cols,
    const int32_t* __restrict__ src_idx, float* __restrict__ dst_cols,
    int32_t* __restrict__ dst_idx, float* __restrict__ psamp, int64_t n, int d)
{
    constexpr int kR = kChunk / kBlock;  // 16 elements per thread
    __shared__ uint16_t perm[kChunk];
    __shared__ uint32_t stage[kChunk];
    __shared__ uint32_t cnt[kR][kWavesPerBlock];
    __shared__ uint32_t pre[kR * kWavesPerBlock + 1];
    // per child: sample slot (-1: none), first sample rank in the run, run
    // length, child count, child position of the run's first point
    __shared__ int ps_par[2][5];
    const int b = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
    if (b >= L.cnt[1]) return;
    const int node = L.bnode[b];
    const int64_t start = L.start[node], c = L.count[node];
    const int64_t beg = L.bbeg[b];
    const int len = (int)(beg + kChunk < c ? kChunk : c - beg);
    const int dim = dimv[node];
    const float split = splitv[node];
    const int64_t nl = n_left[node];
    const int64_t lefts_before = blk_off[b];
    const int64_t base_l = start + lefts_before;
    const int64_t base_r = start + nl + (beg - lefts_before);
    const int64_t src0 = start + beg;
    // flags in element order e = 256 r + t; per (r, wave) ballot counts
    uint64_t lmask[kR];
    const float* key = src_cols + (int64_t)(dim >= 0 ? dim : 0) * n + src0;
    float kv[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {  // every key load in flight at once, clamped in range
        const int e = kBlock * r + t;
        kv[r] = key[e < len ? e : len - 1];
    }
    // kLarge: the split column (column 0 for a node that stays whole) is
    // moved first, staged here from the key loads
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int e = kBlock * r + t;
        const bool ok = e < len;
        const bool f = ok && (dim < 0 || kv[r] < split);
        lmask[r] = __ballot(f);
        if (lane == 0) cnt[r][w] = (uint32_t)__popcll(lmask[r]);
        if (kLarge && ok) stage[e] = __float_as_uint(kv[r]);
    }
    __syncthreads();
    // exclusive prefix of the 64 (r, wave) counts, in element order
    if (w == 0) {
        const uint32_t v = cnt[lane >> 2][lane & 3];
        uint32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        pre[lane] = x - v;
        if (lane == 63) pre[64] = x;
    }
    __syncthreads();
    const uint32_t nl_chunk = pre[64];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const uint32_t before = pre[r * kWavesPerBlock + w];
        const int e = kBlock * r + t;
        if (e < len) {
            const bool f = (lmask[r] >> lane) & 1;
            const uint32_t lb = before + lanes_below(lmask[r]);  // lefts before e
            const uint32_t slot = f ? lb : nl_chunk + (uint32_t)e - lb;
            perm[slot] = (uint16_t)e;
        }
    }
    if (kLarge && t < 2) {
        // the children's sample ranks from j0 on lie in this chunk's runs: run
        // k holds child positions p0 .. p0 + rlen - 1 at output slots from
        // k ? nl_chunk : 0 (the sample position of rank j is
        // floor((2j + 1) c' / 2048), s = 1024); thread k takes child k
        const int k = t;
        const int cc = k ? (int)(c - nl) : (int)nl;
        const int p0 = (int)(k ? beg - lefts_before : lefts_before);
        const int rl = k ? len - (int)nl_chunk : (int)nl_chunk;
        const int sl = dim >= 0 ? cslot[2 * (int64_t)node + k] : -1;
        const bool on = sl >= 0 && sl < ps_cap && cc >= kPreSampleMin && rl > 0;
        int j0 = 0;
        if (on) {  // the smallest j with (2j + 1) c' >= 2048 p0
            const int64_t num = 2 * (int64_t)kSampleMax * p0 - cc, den = 2 * (int64_t)cc;
            if (num > 0) {
                int64_t j = (int64_t)ceil((double)num / (double)den);  // exact after the fix-ups
                if (j * den < num) ++j;
                if (j > 0 && (j - 1) * den >= num) --j;
                j0 = (int)j;
            }
        }
        ps_par[k][0] = on ? sl : -1;
        ps_par[k][1] = j0;
        ps_par[k][2] = rl;
        ps_par[k][3] = cc;
        ps_par[k][4] = p0;
    }
    __syncthreads();
    // columns, each staged in LDS and then written as the left and right
    // runs; the last pass moves the index column (column d).  The next
    // column's loads are issued before the barrier so that their latency
    // overlaps this column's writes.
    uint32_t nxt[kR];
    if constexpr (kLarge) {
        // pass 0 the split column kc (staged above), passes 1 .. d - 1 the
        // other coordinate columns in order
        const int kc = dim >= 0 ? dim : 0;
        int col = kc, ncol = kc == 0 ? 1 : 0;  // this pass's column and the next one's
        for (int it = 0; it <= d; ++it, col = ncol, ncol += ncol + 1 == kc ? 2 : 1) {
            uint32_t* dstw = col < d
                ? reinterpret_cast<uint32_t*>(dst_cols + (int64_t)col * n)
                : reinterpret_cast<uint32_t*>(dst_idx);
            if (it > 0) {
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    const int e = kBlock * r + t;
                    if (e < len) stage[e] = nxt[r];
                }
            }
            if (it < d) {
                const uint32_t* srcw = ncol < d
                    ? reinterpret_cast<const uint32_t*>(src_cols + (int64_t)ncol * n)
                    : reinterpret_cast<const uint32_t*>(src_idx);
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    const int e = kBlock * r + t;
                    nxt[r] = srcw[src0 + (e < len ? e : len - 1)];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int i = kBlock * r + t;
                if (i < len) {
                    const int64_t dst =
                        i < (int)nl_chunk ? base_l + i : base_r + (i - (int)nl_chunk);
                    dstw[dst] = stage[perm[i]];
                }
            }
            // the children's samples (the loop bodies stay rolled: unrolled, they
            // need more registers)
            if (col < d) {
#pragma unroll 1
                for (int k = 0; k < 2; ++k) {  // block-uniform values, in scalar registers
                    const int sl = __builtin_amdgcn_readfirstlane(ps_par[k][0]);
                    if (sl < 0) continue;
                    uint32_t* ps = reinterpret_cast<uint32_t*>(psamp) +
                                   ((int64_t)sl * d + col) * kSampleMax;
                    const int i0 = k == 0 ? 0 : __builtin_amdgcn_readfirstlane((int)nl_chunk);
                    const int rlen = __builtin_amdgcn_readfirstlane(ps_par[k][2]);
                    const uint32_t cc = (uint32_t)__builtin_amdgcn_readfirstlane(ps_par[k][3]);
                    const int p0 = __builtin_amdgcn_readfirstlane(ps_par[k][4]);
#pragma unroll 1
                    for (int j = __builtin_amdgcn_readfirstlane(ps_par[k][1]) + t; j < kSampleMax;
                         j += kBlock) {
                        // (2j + 1) c' >> 11 from the 64-bit product's two halves
                        const uint32_t a = 2u * (uint32_t)j + 1u;
                        const uint32_t pos = (__umulhi(a, cc) << 21) | ((a * cc) >> 11);
                        const int q = (int)pos - p0;
                        if (q >= rlen) break;
                        ps[j] = stage[perm[i0 + q]];
                    }
                }
            }
            __syncthreads();
        }
    } else {
        // the columns in order, column 0 loaded here
        {
            const uint32_t* srcw = d > 0 ? reinterpret_cast<const uint32_t*>(src_cols)
                                         : reinterpret_cast<const uint32_t*>(src_idx);
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int e = kBlock * r + t;
                nxt[r] = srcw[src0 + (e < len ? e : len - 1)];
            }
        }
        for (int col = 0; col <= d; ++col) {
            uint32_t* dstw = col < d
                ? reinterpret_cast<uint32_t*>(dst_cols + (int64_t)col * n)
                : reinterpret_cast<uint32_t*>(dst_idx);
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int e = kBlock * r + t;
                if (e < len) stage[e] = nxt[r];
            }
            if (col < d) {
                const uint32_t* srcw = col + 1 < d
                    ? reinterpret_cast<const uint32_t*>(src_cols + (int64_t)(col + 1) * n)
                    : reinterpret_cast<const uint32_t*>(src_idx);
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    const int e = kBlock * r + t;
                    nxt[r] = srcw[src0 + (e < len ? e : len - 1)];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int i = kBlock * r + t;
                if (i < len) {
                    const int64_t dst =
                        i < (int)nl_chunk ? base_l + i : base_r + (i - (int)nl_chunk);
                    dstw[dst] = stage[perm[i]];
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// B8-B9: subtree finish, one wavefront per node of at most W points
// ---------------------------------------------------------------------------

// Ordered 32-bit key of a float: equal floats (including -0 and +0) get the
// same key, and key order is float order.
__device__ inline uint32_t float_key(float v)
{
    const uint32_t b = __float_as_uint(v + 0.0f);  // -0 becomes +0
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float key_float(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__device__ inline uint32_t wave_min_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// DPP lane moves inside a row of 16 lanes.  row_ror:w gives lane l the value
// of lane (l + w) mod 16 of its row; row_shl:w gives lane l the value of lane
// l + w (meaningful for l + w < 16).
template <int CTRL>
__device__ inline float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
constexpr int kRowRor = 0x120, kRowShl = 0x100;

// Minimum and maximum over the wavefront of N values at once (order does not
// matter for min/max, so rotations inside rows, then two cross-row swaps).
template <int N>
__device__ inline void wave_minmax(float (&lo)[N], float (&hi)[N])
{
#define KNN_MM_STEP(CTRL)                                         \
    _Pragma("unroll") for (int i = 0; i < N; ++i)                 \
    {                                                             \
        lo[i] = fminf(lo[i], dpp_f<CTRL>(lo[i]));                 \
        hi[i] = fmaxf(hi[i], dpp_f<CTRL>(hi[i]));                 \
    }
    KNN_MM_STEP(kRowRor + 8)
    KNN_MM_STEP(kRowRor + 4)
    KNN_MM_STEP(kRowRor + 2)
    KNN_MM_STEP(kRowRor + 1)
#undef KNN_MM_STEP
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            lo[i] = fminf(lo[i], __shfl_xor(lo[i], o));
            hi[i] = fmaxf(hi[i], __shfl_xor(hi[i], o));
        }
    }
}

// Cross-lane part of the pairwise tree for N sums at once: a[l] += a[l + w]
// for w = 32, 16, 8, 4, 2, 1 (the last four through DPP); lane 0's value is
// the sum, returned to every lane.
template <int N>
__device__ inline void wave_tree_n(double (&v)[N], double (&out)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + __shfl_down(v[i], 32);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + __shfl_down(v[i], 16);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<kRowShl + 8>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<kRowShl + 4>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<kRowShl + 2>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<kRowShl + 1>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v[i]));
        const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v[i]));
        out[i] = __hiloint2double(hi, lo);
    }
}

// Lane-local part of the pairwise tree (wave_psum's order) for N sums:
// element l + 64 r of sum i is val(i, r), for r < RM; registers r >= R are
// zeros, whose additions are skipped (they would not change the sum), and so
// are the steps of the 1024-wide tree that pair registers at or above RM.
// The first level is formed straight from the values.
template <int N, int RM, class Val>
__device__ inline void lane_tree_n(int R, Val val, double (&out)[N])
{
    if constexpr (RM == 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = val(i, 0);
    } else {
        constexpr int H = RM / 2;
        double a[N][H];
#pragma unroll
        for (int r = 0; r < H; ++r)
#pragma unroll
            for (int i = 0; i < N; ++i)
                a[i][r] = (r + H < R) ? val(i, r) + val(i, r + H) : val(i, r);
#pragma unroll
        for (int h = H / 2; h >= 1; h >>= 1) {
#pragma unroll
            for (int r = 0; r < h; ++r)
                if (r + h < R) {
#pragma unroll
                    for (int i = 0; i < N; ++i) a[i][r] = a[i][r] + a[i][r + h];
                }
        }
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = a[i][0];
    }
}

// The split of a node whose every point is a sample (the histogram rule
// with s = cnt): the value of rank floor(lc/2) of the keys, or the next larger
// value, whichever leaves the count below it closer to lc/2 (ties to the
// smaller value).  The rank is found by a bitwise search over the ordered keys
// (wavefront ballots); key[r] is the key of node point lane + 64 r, for
// r < R, and kmin < kmax are the smallest and largest keys.
template <int RM>
__device__ inline void median_split(const uint32_t (&key)[RM], int R, int lc, int lane,
                                    uint32_t kmin, uint32_t kmax, float& split, int& nl)
{
    const int m = lc >> 1;
    const int hb = 31 - __clz(kmin ^ kmax);
    uint32_t ans = hb >= 31 ? 0u : (kmin & ~((2u << hb) - 1u));
    for (int b = hb; b >= 0; --b) {
        const uint32_t t = ans | ((1u << b) - 1u);
        int cnt = 0;
#pragma unroll
        for (int r = 0; r < RM; ++r)
            if (r < R) cnt += __popcll(__ballot(lane + kWave * r < lc && key[r] <= t));
        if (cnt <= m) ans |= 1u << b;
    }
    int r_lo = 0, r_hi = 0;
    uint32_t kn = 0xffffffffu;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        if (r < R) {
            const bool ok = lane + kWave * r < lc;
            r_lo += __popcll(__ballot(ok && key[r] < ans));
            r_hi += __popcll(__ballot(ok && key[r] <= ans));
            if (ok && key[r] > ans) kn = min(kn, key[r]);
        }
    }
    kn = wave_min_u32(kn);
    const bool ok_star = r_lo > 0, ok_next = r_hi < lc;
    if (ok_star && (!ok_next || (lc - 2 * r_lo) <= (2 * r_hi - lc))) {
        split = key_float(ans);
        nl = r_lo;
    } else {
        split = key_float(kn);
        nl = r_hi;
    }
}

// Registers per lane of the largest node a finish wavefront handles: the
// subtree limit is 64 * kFinishMaxR<D> points (512 up to 8 dimensions, else
// 256).  The finish is latency-bound, so this limit is set by occupancy: a
// 1024-point subtree needs twice the LDS and, for its 16-row nodes, about
// twice the registers, which halves the wavefronts a SIMD can switch between.
constexpr int finish_rows(int d) { return d <= 8 ? 8 : 4; }
template <int D>
constexpr int kFinishMaxR = finish_rows(D);
// Rows per lane of a subtree node split straight from HBM: subtrees of up to
// 64 * kGlobalRows points are handed to the finish, and their nodes above the
// LDS tile are split in registers, one level per pass over the node.
constexpr int kGlobalRows = 16;
// Rows of 64 points in the largest LDS tile (any dimension).
constexpr int kTileRows = 8;
// Stack entry flag of a node whose points are in a HBM buffer, not in LDS.
constexpr int kInHbm = 1 << 17;

// Context of one wavefront's subtree build.
struct FinishCtx {
    float* X;      // LDS tile: coordinates [D][W]
    int32_t* I;    // LDS tile: input indices [W]
    uint16_t* pm;  // LDS tile: permutation [W], partitioned in place
    int4* stack;
    int W, leaf, max_depth, depth0;
    int64_t gs;    // HBM position of tile element 0
    NodeRec* trec;
    float* tb;
    float* pts;
    int lane;
};

// Process one node of RM or fewer registers per lane (lc <= 64 RM points):
// its box, its split (or bucket rows), the stable partition, and the pushes
// of its children.  Returns the number of stack entries written.
template <int D, int RM>
__device__ int finish_node(const FinishCtx& cx, int id, int ls, int lc, int dep, int sp,
                           int& nloc, int& maxdep, bool& bad)
{
    constexpr int D2 = 2 * D;
    float* X = cx.X;
    uint16_t* pm = cx.pm;
    int4* stack = cx.stack;
    const int W = cx.W, leaf = cx.leaf, max_depth = cx.max_depth, lane = cx.lane;
    const int64_t gs = cx.gs;
    NodeRec* trec = cx.trec;
    float* tb = cx.tb;
    float* pts = cx.pts;
    const int R = (lc + kWave - 1) / kWave;
    // the node's whole permutation slice is read into registers before the
    // partition writes it back in place
    int p[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {  // unconditional LDS loads, clamped in range
        const int j = lane + kWave * r;
        const int q = pm[ls + (j < lc ? j : lc - 1)];
        p[r] = (r < R && j < lc) ? q : 0;
    }
    const bool small = lc <= leaf;
    // box, and the FP64 variance of every dimension (all node points),
    // DC dimensions at a time so their reductions overlap (one at a time for
    // the 8-row nodes, whose registers would otherwise set the occupancy)
    constexpr int DC = RM >= 8 ? 1 : (D <= 3 ? D : (D <= 8 ? 2 : 1));
    float lo_d[D], hi_d[D];
    double bestV = -1.0;
    int best = 0;
#pragma unroll
    for (int d0 = 0; d0 < D; d0 += DC) {
        float v[DC][RM];
        float lo[DC], hi[DC];
#pragma unroll
        for (int i = 0; i < DC; ++i) {
            lo[i] = INFINITY;
            hi[i] = -INFINITY;
            if (d0 + i < D) {
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    const int j = lane + kWave * r;
                    const bool ok = r < R && j < lc;
                    const float xv = X[(d0 + i) * W + p[r]];  // p[r] = 0 past the end
                    v[i][r] = ok ? xv : 0.0f;
                    if (ok) {
                        lo[i] = fminf(lo[i], v[i][r]);
                        hi[i] = fmaxf(hi[i], v[i][r]);
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < RM; ++r) v[i][r] = 0.0f;
            }
        }
        wave_minmax<DC>(lo, hi);
#pragma unroll
        for (int i = 0; i < DC; ++i)
            if (d0 + i < D) {
                lo_d[d0 + i] = lo[i];
                hi_d[d0 + i] = hi[i];
            }
        if (!small) {
            double part[DC], S[DC], V[DC];
            // v is zero where there is no point
            lane_tree_n<DC, RM>(R, [&](int i, int r) { return (double)v[i][r]; }, part);
            wave_tree_n<DC>(part, S);
            const double dlc = (double)lc;
            lane_tree_n<DC, RM>(
                R,
                [&](int i, int r) {
                    const double wv = dlc * (double)v[i][r] - S[i];
                    return (lane + kWave * r < lc) ? wv * wv : 0.0;
                },
                part);
            wave_tree_n<DC>(part, V);
#pragma unroll
            for (int i = 0; i < DC; ++i)
                if (d0 + i < D && V[i] > bestV) {
                    bestV = V[i];
                    best = d0 + i;
                }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            tb[(int64_t)id * D2 + dd] = lo_d[dd];
            tb[(int64_t)id * D2 + D + dd] = hi_d[dd];
        }
    }
    if (small || !(bestV > 0.0)) {  // bucket (or identical points): final rows
        if (lane == 0) {
            trec[id].a = (int32_t)(gs + ls);
            trec[id].split = 0.0f;
            trec[id].dim = -lc;
        }
        for (int j = lane; j < lc; j += kWave) {
            const int q = pm[ls + j];
            const int64_t row = (gs + ls + j) * (D + 1);
#pragma unroll
            for (int dd = 0; dd < D; ++dd) pts[row + dd] = X[dd * W + q];
            pts[row + D] = __int_as_float(cx.I[q]);
        }
        return 0;
    }
    // rank floor(lc/2) of the best dimension by a bitwise search on keys
    float v[RM];
    uint32_t key[RM];
    float blo = lo_d[0], bhi = hi_d[0];
#pragma unroll
    for (int dd = 1; dd < D; ++dd) {
        blo = best == dd ? lo_d[dd] : blo;
        bhi = best == dd ? hi_d[dd] : bhi;
    }
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int j = lane + kWave * r;
        const bool ok = r < R && j < lc;
        const float xv = X[best * W + p[r]];
        v[r] = ok ? xv : 0.0f;
        key[r] = ok ? float_key(v[r]) : 0xffffffffu;
    }
    float split;
    int nl;
    median_split<RM>(key, R, lc, lane, float_key(blo), float_key(bhi), split, nl);
    // stable partition, in place
    int run_l = 0, run_r = 0;
    int pos0 = 0;  // new position of this lane's point of row 0
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        if (r < R) {
            const bool ok = lane + kWave * r < lc;
            const bool f = ok && v[r] < split;
            const uint64_t bl = __ballot(f), bv = __ballot(ok);
            if (ok) {
                const int dst = f ? ls + run_l + (int)lanes_below(bl)
                                  : ls + nl + run_r + (int)lanes_below(bv & ~bl);
                pm[dst] = (uint16_t)p[r];
                if (r == 0) pos0 = dst;
            }
            run_l += __popcll(bl);
            run_r += __popcll(bv & ~bl);
        }
    }
    const int L = nloc, Rc = nloc + 1;
    nloc += 2;
    if constexpr (RM == 1 && D <= 4) {  // (the 4D box values fit the registers)
        if (nl <= leaf && lc - nl <= leaf) {
            // both children are buckets: close them here, one point per lane
            // (each lane's point goes to row pos0 of the packed order), with
            // the two boxes reduced together
            if (cx.depth0 + dep + 1 > max_depth) bad = true;
            if (dep + 1 > maxdep) maxdep = dep + 1;
            const bool ok = lane < lc;
            const bool f = ok && v[0] < split;
            float x[D], lo[2 * D], hi[2 * D];
#pragma unroll
            for (int dd = 0; dd < D; ++dd) {
                x[dd] = X[dd * W + p[0]];
                lo[dd] = ok && f ? x[dd] : INFINITY;
                hi[dd] = ok && f ? x[dd] : -INFINITY;
                lo[D + dd] = ok && !f ? x[dd] : INFINITY;
                hi[D + dd] = ok && !f ? x[dd] : -INFINITY;
            }
            wave_minmax<2 * D>(lo, hi);
            if (ok) {
                const int64_t row = (gs + pos0) * (D + 1);
#pragma unroll
                for (int dd = 0; dd < D; ++dd) pts[row + dd] = x[dd];
                pts[row + D] = __int_as_float(cx.I[p[0]]);
            }
            if (lane == 0) {
                trec[id].a = L;
                trec[id].split = split;
                trec[id].dim = best;
                NodeRec cl, cr;
                cl.a = (int32_t)(gs + ls);
                cl.parent = id;
                cl.split = 0.0f;
                cl.dim = -nl;
                cr.a = (int32_t)(gs + ls + nl);
                cr.parent = id;
                cr.split = 0.0f;
                cr.dim = -(lc - nl);
                trec[L] = cl;
                trec[Rc] = cr;
#pragma unroll
                for (int dd = 0; dd < D; ++dd) {
                    tb[(int64_t)L * D2 + dd] = lo[dd];
                    tb[(int64_t)L * D2 + D + dd] = hi[dd];
                    tb[(int64_t)Rc * D2 + dd] = lo[D + dd];
                    tb[(int64_t)Rc * D2 + D + dd] = hi[D + dd];
                }
            }
            wave_sync();
            return 0;
        }
    }
    if (cx.depth0 + dep + 1 > max_depth || sp + 2 > kStack) bad = true;
    if (lane == 0) {
        trec[id].a = L;
        trec[id].split = split;
        trec[id].dim = best;
        trec[L].parent = id;
        trec[Rc].parent = id;
        if (!bad) {
            const int wd = dep + 1;
            const int4 lft = make_int4(L, ls, nl, wd);
            const int4 rgt = make_int4(Rc, ls + nl, lc - nl, wd);
            if (nl <= lc - nl) {  // smaller child next keeps the stack shallow
                stack[sp] = rgt;
                stack[sp + 1] = lft;
            } else {
                stack[sp] = lft;
                stack[sp + 1] = rgt;
            }
        }
    }
    wave_sync();
    return bad ? 0 : 2;
}

// Split one subtree node of more points than the LDS tile holds, straight
// from a HBM buffer pair: its lc <= 64 * kGlobalRows points sit at
// [gs + ls, gs + ls + lc) of columns scol / indices sidx, node order; the
// stable partition goes to the same range of dcol / didx (the other buffer of
// the ping-pong pair, which no other subtree uses there).  The box, the split
// dimension (FP64 variance, the same pairwise tree as finish_node), the split
// (median_split) and the child records are those of finish_node; a node that
// is a bucket writes its packed rows from the buffer.  Returns the number of
// stack entries written (its children, both marked kInHbm for the other
// buffer).
template <int D>
__device__ int finish_global(const FinishCtx& cx, const float* __restrict__ scol,
                             const int32_t* __restrict__ sidx, float* __restrict__ dcol,
                             int32_t* __restrict__ didx, int64_t n, int id, int ls, int lc,
                             int dep, int g, int sp, int& nloc, bool& bad)
{
    constexpr int RG = kGlobalRows;
    constexpr int D2 = 2 * D;
    const int lane = cx.lane;
    const int64_t s0 = cx.gs + ls;
    const int R = (lc + kWave - 1) / kWave;
    const bool small = lc <= cx.leaf;
    double bestV = -1.0;
    int best = 0;
    float blo = 0.0f, bhi = 0.0f;
    // one dimension per pass, not unrolled (the registers of this path count
    // against the whole kernel's occupancy), with the next dimension's rows
    // in flight meanwhile; whole rows are read (the buffers have a tail)
    float vn[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) vn[r] = r < R ? scol[s0 + lane + kWave * r] : 0.0f;
#pragma unroll 1
    for (int dd = 0; dd < D; ++dd) {
        float v[RG];
        float lo[1] = {INFINITY}, hi[1] = {-INFINITY};
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const bool ok = lane + kWave * r < lc;
            v[r] = ok ? vn[r] : 0.0f;
            lo[0] = fminf(lo[0], ok ? vn[r] : INFINITY);
            hi[0] = fmaxf(hi[0], ok ? vn[r] : -INFINITY);
        }
        if (dd + 1 < D) {
            const float* col = scol + (int64_t)(dd + 1) * n + s0;
#pragma unroll
            for (int r = 0; r < RG; ++r) vn[r] = r < R ? col[lane + kWave * r] : 0.0f;
        }
        wave_minmax<1>(lo, hi);
        if (lane == 0) {
            cx.tb[(int64_t)id * D2 + dd] = lo[0];
            cx.tb[(int64_t)id * D2 + D + dd] = hi[0];
        }
        if (!small) {
            double part[1], S[1], V[1];
            lane_tree_n<1, RG>(R, [&](int, int r) { return (double)v[r]; }, part);
            wave_tree_n<1>(part, S);
            const double dlc = (double)lc;
            lane_tree_n<1, RG>(
                R,
                [&](int, int r) {
                    const double wv = dlc * (double)v[r] - S[0];
                    return (lane + kWave * r < lc) ? wv * wv : 0.0;
                },
                part);
            wave_tree_n<1>(part, V);
            if (V[0] > bestV) {
                bestV = V[0];
                best = dd;
                blo = lo[0];
                bhi = hi[0];
            }
        }
    }
    if (small || !(bestV > 0.0)) {  // bucket (or identical points): final rows
        if (lane == 0) {
            cx.trec[id].a = (int32_t)s0;
            cx.trec[id].split = 0.0f;
            cx.trec[id].dim = -lc;
        }
        for (int j = lane; j < lc; j += kWave) {
            const int64_t row = (s0 + j) * (D + 1);
#pragma unroll
            for (int dd = 0; dd < D; ++dd) cx.pts[row + dd] = scol[(int64_t)dd * n + s0 + j];
            cx.pts[row + D] = __int_as_float(sidx[s0 + j]);
        }
        return 0;
    }
    uint32_t key[RG];
    {
        const float* col = scol + (int64_t)best * n + s0;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const int j = lane + kWave * r;
            const float x = r < R ? col[j] : 0.0f;
            key[r] = j < lc ? float_key(x) : 0xffffffffu;
        }
    }
    float split;
    int nl;
    median_split<RG>(key, R, lc, lane, float_key(blo), float_key(bhi), split, nl);
    // destinations of the stable partition (left block, then right block);
    // key order is value order, so the test runs on the keys
    const uint32_t ks = float_key(split);
    int dst[RG];
    int run_l = 0, run_r = 0;
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        dst[r] = 0;
        if (r < R) {
            const bool ok = lane + kWave * r < lc;
            const bool f = ok && key[r] < ks;
            const uint64_t bl = __ballot(f), bv = __ballot(ok);
            dst[r] = f ? run_l + (int)lanes_below(bl) : nl + run_r + (int)lanes_below(bv & ~bl);
            run_l += __popcll(bl);
            run_r += __popcll(bv & ~bl);
        }
    }
    // the D coordinate arrays and the index array, PA at a time (two fit the
    // registers of the low dimensions only)
    constexpr int PA = D <= 3 ? 2 : 1;
#pragma unroll 1
    for (int d0 = 0; d0 <= D; d0 += PA) {
        float t[PA][RG];
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int dd = d0 + i;
            if (dd <= D) {
                const float* src = dd < D ? scol + (int64_t)dd * n + s0
                                          : reinterpret_cast<const float*>(sidx + s0);
#pragma unroll
                for (int r = 0; r < RG; ++r) t[i][r] = r < R ? src[lane + kWave * r] : 0.0f;
            }
        }
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int dd = d0 + i;
            if (dd <= D) {
                float* out = dd < D ? dcol + (int64_t)dd * n + s0
                                    : reinterpret_cast<float*>(didx + s0);
#pragma unroll
                for (int r = 0; r < RG; ++r)
                    if (r < R && lane + kWave * r < lc) out[dst[r]] = t[i][r];
            }
        }
    }
    const int L = nloc, Rc = nloc + 1;
    nloc += 2;
    if (cx.depth0 + dep + 1 > cx.max_depth || sp + 2 > kStack) bad = true;
    if (lane == 0) {
        cx.trec[id].a = L;
        cx.trec[id].split = split;
        cx.trec[id].dim = best;
        cx.trec[L].parent = id;
        cx.trec[Rc].parent = id;
        if (!bad) {
            const int wd = (dep + 1) | ((g ^ 1) << 16) | kInHbm;
            const int4 lft = make_int4(L, ls, nl, wd);
            const int4 rgt = make_int4(Rc, ls + nl, lc - nl, wd);
            if (nl <= lc - nl) {
                cx.stack[sp] = rgt;
                cx.stack[sp + 1] = lft;
            } else {
                cx.stack[sp] = lft;
                cx.stack[sp + 1] = rgt;
            }
        }
    }
    // the children are read back from HBM by other lanes of this wavefront:
    // wait for the stores (the CU's L1 is coherent for its own stores)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return bad ? 0 : 2;
}

// One wavefront builds the whole subtree of one node of at most 64 *
// kGlobalRows points.  Nodes larger than the LDS tile of W points are split
// in registers straight from HBM (finish_global); a node that fits is loaded
// into the tile and it and its descendants are split there (finish_node).
// Every point is a sample at these sizes, so the histogram rule picks the
// value of rank floor(cnt/2) or the next larger value, whichever has its
// count below closer to cnt/2 (ties to the smaller value); the rank is found
// by a bitwise search over the ordered keys with wavefront ballots.  In LDS
// the index permutation ping-pongs between two arrays, and each bucket's
// packed rows are written as soon as the bucket is final.
template <int D>
__device__ __forceinline__ void finish_subtree(
    int sub, unsigned char* smem, const SubEntry* __restrict__ subs, float* colsA, int32_t* idxA,
    float* colsB, int32_t* idxB, int64_t n, int leaf, int W, int max_depth,
    size_t per_wave, float* __restrict__ pts, NodeRec* __restrict__ tnodes,
    float* __restrict__ tbox, int32_t* __restrict__ sub_nodes, int32_t* __restrict__ err,
    int32_t* __restrict__ depth_seen)
{
    constexpr int D2 = 2 * D;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const SubEntry e = subs[sub];
    const float* cols = e.buf ? colsB : colsA;
    const int32_t* gidx = e.buf ? idxB : idxA;
    const int64_t gs = e.start;
    const int c = e.count;
    NodeRec* trec = tnodes + 2 * gs;
    float* tb = tbox + 2 * gs * D2;

    if (e.leaf_only || c <= leaf) {  // a bucket: box and packed rows straight from HBM
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            float lo = INFINITY, hi = -INFINITY;
            for (int j = lane; j < c; j += kWave) {
                float x = cols[(int64_t)dd * n + gs + j];
                lo = fminf(lo, x);
                hi = fmaxf(hi, x);
            }
            lo = wave_min(lo);
            hi = wave_max(hi);
            if (lane == 0) {
                tb[dd] = lo;
                tb[D + dd] = hi;
            }
        }
        for (int j = lane; j < c; j += kWave) {
            const int64_t row = (gs + j) * (D + 1);
#pragma unroll
            for (int dd = 0; dd < D; ++dd) pts[row + dd] = cols[(int64_t)dd * n + gs + j];
            pts[row + D] = __int_as_float(gidx[gs + j]);
        }
        if (lane == 0) {
            NodeRec r;
            r.a = (int32_t)gs;
            r.parent = -1;
            r.split = 0.0f;
            r.dim = -c;
            trec[0] = r;
            sub_nodes[sub] = 1;
            atomicMax(depth_seen, e.depth0);
        }
        return;
    }

    unsigned char* region = smem + (size_t)w * per_wave;
    float* X = reinterpret_cast<float*>(region);                  // [D][W]
    int32_t* I = reinterpret_cast<int32_t*>(X + (size_t)D * W);   // [W]
    uint16_t* pm = reinterpret_cast<uint16_t*>(I + W);            // [W]
    int4* stack = reinterpret_cast<int4*>(pm + W);                // [kStack]

    if (lane == 0) {
        stack[0] = make_int4(0, 0, c, (e.buf << 16) | kInHbm);
        trec[0].parent = -1;
    }
    wave_sync();
    int sp = 1, nloc = 1, maxdep = 0, errc = KNN_EDEPTH;
    bool bad = false;
    int64_t lbase = gs;  // HBM position of the points now in LDS
    while (sp > 0) {
        const int4 top = stack[--sp];
        const int id = __builtin_amdgcn_readfirstlane(top.x);
        const int lc = __builtin_amdgcn_readfirstlane(top.z);
        const int tw = __builtin_amdgcn_readfirstlane(top.w);
        int ls = __builtin_amdgcn_readfirstlane(top.y);
        const int buf = (tw >> 16) & 1;
        const int dep = tw & 0xffff;
        if (dep > maxdep) maxdep = dep;
        int pushed;
        if (tw & kInHbm) {
            const float* scol = buf ? colsB : colsA;
            const int32_t* sidx = buf ? idxB : idxA;
            if (lc > W) {  // larger than the LDS tile: one split in registers
                if (lc > kWave * kGlobalRows) {
                    bad = true;
                    errc = KNN_EDEVICE;
                    break;
                }
                FinishCtx hctx{X, I, pm, stack, W, leaf, max_depth, e.depth0, gs, trec, tb, pts,
                               lane};
                pushed = finish_global<D>(hctx, scol, sidx, buf ? colsA : colsB,
                                          buf ? idxA : idxB, n, id, ls, lc, dep, buf, sp, nloc,
                                          bad);
                if (bad) break;
                sp += pushed;
                continue;
            }
            // the node fits the tile: load it (whole rows, every load of an
            // array in flight at once; the buffers have a tail), then split
            // it and its descendants, all above it on the stack, in LDS
            wave_sync();
            const int R = (lc + kWave - 1) / kWave;
            const int64_t s0 = gs + ls;
#pragma unroll
            for (int dd = 0; dd <= D; ++dd) {
                const float* src = dd < D ? scol + (int64_t)dd * n + s0
                                          : reinterpret_cast<const float*>(sidx + s0);
                float* dst = dd < D ? X + dd * W : reinterpret_cast<float*>(I);
                float t[kTileRows];
#pragma unroll
                for (int r = 0; r < kTileRows; ++r) t[r] = r < R ? src[lane + kWave * r] : 0.0f;
#pragma unroll
                for (int r = 0; r < kTileRows; ++r)
                    if (r < R) dst[lane + kWave * r] = t[r];
            }
#pragma unroll
            for (int r = 0; r < kTileRows; ++r)
                if (r < R) pm[lane + kWave * r] = (uint16_t)(lane + kWave * r);
            wave_sync();
            lbase = s0;
            ls = 0;
        }
        const int R = (lc + kWave - 1) / kWave;
        FinishCtx ctx{X, I, pm, stack, W, leaf, max_depth, e.depth0, lbase, trec, tb, pts, lane};
        if (R <= 1) pushed = finish_node<D, 1>(ctx, id, ls, lc, dep, sp, nloc, maxdep, bad);
        else if (R <= 2) pushed = finish_node<D, 2>(ctx, id, ls, lc, dep, sp, nloc, maxdep, bad);
        else if (R <= 4 || kFinishMaxR<D> == 4)
            pushed = finish_node<D, 4>(ctx, id, ls, lc, dep, sp, nloc, maxdep, bad);
        else pushed = finish_node<D, 8>(ctx, id, ls, lc, dep, sp, nloc, maxdep, bad);
        if (bad) break;
        sp += pushed;
    }
    if (bad) {
        if (lane == 0) atomicExch(err, errc);
        return;
    }
    if (lane == 0) {
        sub_nodes[sub] = nloc;
        atomicMax(depth_seen, e.depth0 + maxdep);
    }
}

// One wavefront per subtree, subtrees sub0 + (wavefront index) of the grid;
// with kStride, also every grid-sized stride beyond (the tail of a launch
// whose grid was fixed before the count was known).  The count is n_sub, or
// *n_sub_dev when that is set.  The single-subtree form keeps the register
// count of a body without a loop around it (occupancy 4).
template <int D, bool kStride>
__global__ __launch_bounds__(kBlock) void k_finish(
    const SubEntry* __restrict__ subs, int32_t sub0, int32_t n_sub,
    const int32_t* __restrict__ n_sub_dev, float* colsA, int32_t* idxA, float* colsB,
    int32_t* idxB, int64_t n, int leaf, int W, int max_depth, size_t per_wave,
    float* __restrict__ pts, NodeRec* __restrict__ tnodes, float* __restrict__ tbox,
    int32_t* __restrict__ sub_nodes, int32_t* __restrict__ err, int32_t* __restrict__ depth_seen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int total = n_sub_dev ? __builtin_amdgcn_readfirstlane(*n_sub_dev) : n_sub;
    // only wavefront-level synchronization below
    int sub = sub0 + blockIdx.x * kWavesPerBlock + w;
    if constexpr (kStride) {
        for (; sub < total; sub += gridDim.x * kWavesPerBlock)
            finish_subtree<D>(sub, smem, subs, colsA, idxA, colsB, idxB, n, leaf, W, max_depth,
                              per_wave, pts, tnodes, tbox, sub_nodes, err, depth_seen);
    } else {
        if (sub < total)
            finish_subtree<D>(sub, smem, subs, colsA, idxA, colsB, idxB, n, leaf, W, max_depth,
                              per_wave, pts, tnodes, tbox, sub_nodes, err, depth_seen);
    }
}

// Final ids: subtree root keeps its level-pass id, local node j >= 1 becomes
// sub_base + j - 1.
__global__ __launch_bounds__(kBlock) void k_compact(const SubEntry* __restrict__ subs,
                                                    int32_t n_sub,
                                                    const int32_t* __restrict__ n_sub_dev,
                                                    const int32_t* __restrict__ sub_nodes,
                                                    const int32_t* __restrict__ sub_base,
                                                    const NodeRec* __restrict__ tnodes,
                                                    const float* __restrict__ tbox, int d,
                                                    NodeRec* __restrict__ nodes,
                                                    float* __restrict__ bbox)
{
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int total = n_sub_dev ? __builtin_amdgcn_readfirstlane(*n_sub_dev) : n_sub;
    for (int sub = blockIdx.x * kWavesPerBlock + w; sub < total; sub += gridDim.x * kWavesPerBlock) {
    const SubEntry e = subs[sub];
    const int cnt = sub_nodes[sub];
    const int base = sub_base[sub];
    const int64_t gs = e.start;
    const int D2 = 2 * d;
    auto gid = [&](int j) { return j == 0 ? e.node_id : base + j - 1; };
    for (int j = lane; j < cnt; j += kWave) {
        NodeRec r = tnodes[2 * gs + j];
        NodeRec o;
        o.parent = j == 0 ? e.parent : gid(r.parent);
        o.split = r.split;
        o.dim = r.dim;
        o.a = r.dim >= 0 ? gid(r.a) : r.a;
        const int g = gid(j);
        nodes[g] = o;
        for (int t = 0; t < D2; ++t) bbox[(int64_t)g * D2 + t] = tbox[(2 * gs + j) * D2 + t];
    }
    }
}

// Boxes of the level-pass nodes of one depth, whose ids form the range
// rng[0] .. rng[1]: union of the two children's boxes.  Run from the deepest
// level up; subtree roots in the range already hold their box (recomputing
// it from their children gives the same tight box).
__global__ void k_bbox_up(const int32_t* __restrict__ rng, const NodeRec* __restrict__ nodes,
                          float* __restrict__ bbox, int d)
{
    const int v = rng[0] + blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= rng[1]) return;
    if (nodes[v].dim < 0) return;
    const int L = nodes[v].a;
    const int D2 = 2 * d;
    for (int t = 0; t < d; ++t) {
        bbox[(int64_t)v * D2 + t] = fminf(bbox[(int64_t)L * D2 + t], bbox[(int64_t)(L + 1) * D2 + t]);
        bbox[(int64_t)v * D2 + d + t] =
            fmaxf(bbox[(int64_t)L * D2 + d + t], bbox[(int64_t)(L + 1) * D2 + d + t]);
    }
}

// ---------------------------------------------------------------------------
// B7: level bookkeeping on the device
// ---------------------------------------------------------------------------
constexpr int kPlanBlock = 1024;

// Exclusive scan over the level's nodes of the plan counters (planv ->
// planx), by one block; the totals give the next level's sizes and advance
// the id and subtree counters.  Every position comes from a prefix sum, so
// ids and list order do not depend on thread timing.
// Exclusive scan of the per-node plan values, in two kernels: each block of
// kPlanBlock nodes scans its own (coalesced, one node per thread) and leaves
// its totals in pblk; k_plan_top scans the block totals, and k_plan_write
// adds a node's block offset to its in-block prefix.
__global__ __launch_bounds__(kPlanBlock) void k_plan_local(
    Level cur, const int32_t* __restrict__ planv, int32_t* __restrict__ planx,
    int32_t* __restrict__ pblk, int32_t* __restrict__ g)
{
    __shared__ int wsum[kPlanBlock / 64][kPlanVals];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int nn = cur.cnt[0];
    const int i = blockIdx.x * kPlanBlock + t;
    if (blockIdx.x * kPlanBlock >= nn) return;  // block-uniform
    int v[kPlanVals] = {};
    unsigned long long pts = 0;  // points this level partitions (profiling counter)
    if (i < nn) {
#pragma unroll
        for (int k = 0; k < kPlanVals; ++k) v[k] = planv[(int64_t)i * kPlanStride + k];
        pts = (unsigned long long)cur.count[i];
    }
    for (int o = 32; o > 0; o >>= 1) pts += __shfl_xor(pts, o);
    if (lane == 0 && pts) atomicAdd(reinterpret_cast<unsigned long long*>(g + G_MOVED), pts);
    int x[kPlanVals];
#pragma unroll
    for (int k = 0; k < kPlanVals; ++k) x[k] = v[k];
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int k = 0; k < kPlanVals; ++k) {
            const int y = __shfl_up(x[k], o);
            if (lane >= o) x[k] += y;
        }
    }
    if (lane == 63)
#pragma unroll
        for (int k = 0; k < kPlanVals; ++k) wsum[w][k] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPlanVals; ++k) {
        int base = 0, all = 0;
        for (int j = 0; j < kPlanBlock / 64; ++j) {
            if (j < w) base += wsum[j][k];
            all += wsum[j][k];
        }
        if (i < nn) planx[(int64_t)i * kPlanStride + k] = base + x[k] - v[k];
        if (t == 0) pblk[(int64_t)blockIdx.x * kPlanStride + k] = all;
    }
}

__global__ __launch_bounds__(kPlanBlock) void k_plan_top(
    Level cur, Level nxt, int32_t* __restrict__ pblk, int32_t* __restrict__ g,
    int32_t* __restrict__ rng, int level, int64_t big_cap, int64_t sub_cap, int64_t nn_cap,
    int64_t nb_cap, int64_t nbh_cap, int64_t ps_cap)
{
    __shared__ int wsum[kPlanBlock / 64][kPlanVals];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int nblk = (cur.cnt[0] + kPlanBlock - 1) / kPlanBlock;
    int carry[kPlanVals] = {};
    for (int b0 = 0; b0 < nblk; b0 += kPlanBlock) {  // exclusive scan of the block totals
        const int b = b0 + t;
        int v[kPlanVals], x[kPlanVals];
#pragma unroll
        for (int k = 0; k < kPlanVals; ++k) {
            v[k] = b < nblk ? pblk[(int64_t)b * kPlanStride + k] : 0;
            x[k] = v[k];
        }
        for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
            for (int k = 0; k < kPlanVals; ++k) {
                const int y = __shfl_up(x[k], o);
                if (lane >= o) x[k] += y;
            }
        }
        if (lane == 63)
#pragma unroll
            for (int k = 0; k < kPlanVals; ++k) wsum[w][k] = x[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPlanVals; ++k) {
            int base = 0, all = 0;
            for (int j = 0; j < kPlanBlock / 64; ++j) {
                if (j < w) base += wsum[j][k];
                all += wsum[j][k];
            }
            if (b < nblk) pblk[(int64_t)b * kPlanStride + k] = carry[k] + base + x[k] - v[k];
            carry[k] += all;
        }
        __syncthreads();
    }
    if (t == 0) {
        const int* tot = carry;
        const int base_id = g[G_NEXT_ID], base_sub = g[G_NSUB];
        g[G_BASE_ID] = base_id;
        g[G_BASE_SUB] = base_sub;
        g[G_NEXT_ID] = base_id + 2 * tot[0];
        g[G_NSUB] = base_sub + tot[2];
        nxt.cnt[0] = tot[1];
        nxt.cnt[1] = tot[3];
        nxt.cnt[2] = tot[4];
        g[G_LEVEL_NODES] = tot[1];
        rng[2 * (level + 1)] = base_id;
        rng[2 * (level + 1) + 1] = base_id + 2 * tot[0];
        if (base_id + 2 * (int64_t)tot[0] > big_cap || base_sub + (int64_t)tot[2] > sub_cap ||
            tot[1] > nn_cap || tot[3] > nb_cap || tot[4] > nbh_cap || tot[5] > ps_cap) {
            atomicExch(&g[G_ERR], kErrOverflow);
            nxt.cnt[0] = nxt.cnt[1] = nxt.cnt[2] = 0;  // nothing more is written
            g[G_LEVEL_NODES] = 0;
        }
    }
}

// One thread per node of the level: the split node's record (children get
// ids L and L+1, L = base + 2 * (split nodes before it)), its children in
// the next level's node list (with their pre-gathered sample slots when the
// partition of this level writes them, also left in cslot for it) or in the
// subtree list, and nodes whose points all coincide as oversized buckets.
__global__ __launch_bounds__(kBlock) void k_plan_write(
    Level cur, Level nxt, const int32_t* __restrict__ dimv, const float* __restrict__ splitv,
    const int32_t* __restrict__ nleft, const int32_t* __restrict__ planx,
    const int32_t* __restrict__ pblk, int leaf, int W, int max_depth, int nbuf,
    NodeRec* __restrict__ big, SubEntry* __restrict__ subs, int32_t* __restrict__ cslot,
    int presample, int32_t* __restrict__ g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cur.cnt[0]) return;
    cslot[2 * (int64_t)i] = cslot[2 * (int64_t)i + 1] = -1;
    if (g[G_ERR] == kErrOverflow) return;
    const int st = cur.start[i], cnt = cur.count[i], id = cur.id[i];
    const int par = cur.parent[i], dep = cur.depth[i], dm = dimv[i];
    int x[kPlanVals];
#pragma unroll
    for (int k = 0; k < kPlanVals; ++k)
        x[k] = planx[(int64_t)i * kPlanStride + k] + pblk[(int64_t)(i / kPlanBlock) * kPlanStride + k];
    const int base_id = g[G_BASE_ID], base_sub = g[G_BASE_SUB];
    if (dm < 0) {  // all points identical: an oversized bucket
        subs[base_sub + x[2]] = SubEntry{st, cnt, id, par, nbuf, 1, dep, 0};
        return;
    }
    const int nl = nleft[i];
    const int L = base_id + 2 * x[0];
    big[id] = NodeRec{L, par, splitv[i], dm};
    if (dep + 1 > max_depth) atomicCAS(&g[G_ERR], 0, KNN_EDEPTH);
    const int cs[2] = {st, st + nl}, cc[2] = {nl, cnt - nl};
    int pos = x[1], b0 = x[3], h0 = x[4], sidx = base_sub + x[2], ps = x[5];
    for (int k = 0; k < 2; ++k) {
        if (needs_level_pass(cc[k], W, leaf)) {
            const int sl = presample && cc[k] >= kPreSampleMin ? ps++ : -1;
            cslot[2 * (int64_t)i + k] = sl;
            nxt.sslot[pos] = sl;
            nxt.start[pos] = cs[k];
            nxt.count[pos] = cc[k];
            nxt.id[pos] = L + k;
            nxt.parent[pos] = id;
            nxt.depth[pos] = dep + 1;
            nxt.blk0[pos] = b0;
            nxt.nblk[pos] = (cc[k] + kChunk - 1) / kChunk;
            nxt.hblk0[pos] = h0;
            b0 += (cc[k] + kChunk - 1) / kChunk;
            h0 += (cc[k] + kHistChunk - 1) / kHistChunk;
            ++pos;
        } else {
            subs[sidx++] = SubEntry{cs[k], cc[k], L + k, id, nbuf, 0, dep + 1, 0};
        }
    }
}

// Block tables of the next level: block b belongs to the node whose first
// block is the largest blk0 <= b (every node has at least one block).
__global__ __launch_bounds__(kBlock) void k_plan_fill(Level nxt)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int nn = nxt.cnt[0], nb = nxt.cnt[1], nbh = nxt.cnt[2];
    for (int tab = 0; tab < 2; ++tab) {
        const int lim = tab ? nbh : nb;
        if (b >= lim) continue;
        const int32_t* first = tab ? nxt.hblk0 : nxt.blk0;
        int lo = 0, hi = nn - 1;  // largest pos with first[pos] <= b
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        if (tab) {
            nxt.hnode[b] = lo;
            nxt.hbeg[b] = (b - first[lo]) * kHistChunk;
        } else {
            nxt.bnode[b] = lo;
            nxt.bbeg[b] = (b - first[lo]) * kChunk;
        }
    }
}

// Int32 words of one Level with the given capacities.
inline size_t level_words(int64_t nn_cap, int64_t nb_cap, int64_t nbh_cap)
{
    return 9 * (size_t)nn_cap + 2 * (size_t)nb_cap + 2 * (size_t)nbh_cap + 4;
}

// The arrays of one Level laid out in level_words() words at p.
inline Level carve_level(int32_t* p, int64_t nn_cap, int64_t nb_cap, int64_t nbh_cap)
{
    Level L{};
    L.start = p; p += nn_cap;
    L.count = p; p += nn_cap;
    L.id = p; p += nn_cap;
    L.parent = p; p += nn_cap;
    L.depth = p; p += nn_cap;
    L.blk0 = p; p += nn_cap;
    L.nblk = p; p += nn_cap;
    L.bnode = p; p += nb_cap;
    L.bbeg = p; p += nb_cap;
    L.hnode = p; p += nbh_cap;
    L.hbeg = p; p += nbh_cap;
    L.hblk0 = p; p += nn_cap;
    L.sslot = p; p += nn_cap;
    L.cnt = p;
    return L;
}

// Device buffers of one Level with the given capacities.
struct LevelMem {
    DevBuf mem;
    Level L{};
    explicit LevelMem(hipStream_t s) : mem(s) {}
    hipError_t alloc(int64_t nn_cap, int64_t nb_cap, int64_t nbh_cap)
    {
        hipError_t e = mem.alloc(sizeof(int32_t) * level_words(nn_cap, nb_cap, nbh_cap));
        if (e != hipSuccess) return e;
        L = carve_level(mem.as<int32_t>(), nn_cap, nb_cap, nbh_cap);
        return hipSuccess;
    }
};

using FinishFn = void (*)(const SubEntry*, int32_t, int32_t, const int32_t*, float*, int32_t*,
                          float*, int32_t*, int64_t, int, int, int, size_t, float*, NodeRec*,
                          float*, int32_t*, int32_t*, int32_t*);

FinishFn finish_for(int d, bool stride = false)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return stride ? k_finish<DD, true> : k_finish<DD, false>;
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4)
        KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
        KNN_DIM_CASE(9) KNN_DIM_CASE(10) KNN_DIM_CASE(11) KNN_DIM_CASE(12)
        KNN_DIM_CASE(13) KNN_DIM_CASE(14) KNN_DIM_CASE(15) KNN_DIM_CASE(16)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
}

inline unsigned blocks_for(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

// The host side of level 0.  Tree t has root node t.  Roots of at most W
// points (or at most a bucket) go straight to the subtree finish; the
// others form level 0, with their block tables.
struct Level0Host {
    std::vector<int32_t> f[8];  // per large root: start, count, id, parent, depth, blk0, nblk, hblk0
    int32_t nb0 = 0, nbh0 = 0;  // partition and histogram blocks of level 0
    std::vector<SubEntry> small;
    std::vector<int32_t> big_roots;
    int64_t largest = 0;
};

Level0Host level0_tables(const int64_t* offsets, int32_t T, int32_t W, int32_t leaf)
{
    Level0Host h;
    for (int32_t r = 0; r < T; ++r) {
        const int64_t c = offsets[r + 1] - offsets[r];
        if (!needs_level_pass((int)c, W, leaf)) {
            h.small.push_back(SubEntry{(int32_t)offsets[r], (int32_t)c, r, -1, 0, 0, 0, 0});
            continue;
        }
        h.big_roots.push_back(r);
        h.largest = std::max(h.largest, c);
        const int32_t nb = (int32_t)((c + kChunk - 1) / kChunk);
        const int32_t nbh = (int32_t)((c + kHistChunk - 1) / kHistChunk);
        const int32_t vals[8] = {(int32_t)offsets[r], (int32_t)c, r, -1, 0, h.nb0, nb, h.nbh0};
        for (int k = 0; k < 8; ++k) h.f[k].push_back(vals[k]);
        h.nb0 += nb;
        h.nbh0 += nbh;
    }
    return h;
}

// Level passes a tree of `largest` points needs when every split halves.
int expected_levels(int64_t largest, int32_t W, int32_t leaf)
{
    int e = 1;
    for (int64_t c = largest; c > W && c > leaf; c = (c + 1) / 2) ++e;
    return e;
}

// Buffers and sizes shared by every level pass of one build.
struct LevelWork {
    float* cols[2];       // SoA coordinates: the pass reads cols[buf], writes cols[buf ^ 1]
    int32_t* idx[2];      // original indices, likewise
    int32_t* dimv;
    float* splitv;
    int32_t* nleft;
    float* samples;
    uint32_t* hist;
    uint16_t* crow;       // per partition block: prefix row of its window counts
    float* psamp;         // pre-gathered samples: [slot][d][1024]
    int32_t* cslot;       // per level node: its two children's sample slots (or -1)
    uint32_t* blk_off;
    int32_t* planv;
    int32_t* planx;
    int32_t* pblk;
    NodeRec* big;         // level-pass node records by id
    SubEntry* subs;       // subtree list
    int32_t* rng;         // id range of each depth's level-pass nodes
    int32_t* g;           // build counters
    int64_t n;
    int d, leaf, W, max_depth;
    int64_t split_block_nodes;
    int64_t nn0;          // nodes of level 0
    int64_t largest;      // points of the largest root
    int64_t nn_cap, nb_cap, nbh_cap, big_cap, sub_cap, ps_cap;
};

// Enqueues one level pass (B1-B7) over the nodes of `cur`, writing the next
// level into `nxt`.  Grids are sized for the largest level possible at this
// depth; the kernels read the actual counts from cur.cnt on the device.  The
// bookkeeping runs before the partition (it needs only the split and the left
// counts), so the partition knows which children take a pre-gathered sample
// and where.
void enqueue_level(const LevelWork& w, const Level& cur, const Level& nxt, int level, int buf,
                   bool prof, hipStream_t st)
{
    const int64_t n = w.n;
    const int64_t nn_l = std::min<int64_t>(level < 40 ? w.nn0 << std::min(level, 40) : w.nn_cap,
                                           w.nn_cap);
    const unsigned g_nn = (unsigned)nn_l;
    const unsigned g_nb = (unsigned)std::min<int64_t>(n / kChunk + nn_l + 1, w.nb_cap);
    const unsigned g_nbh = (unsigned)std::min<int64_t>(n / kHistChunk + nn_l + 1, w.nbh_cap);
    const float* src = w.cols[buf];
    const int32_t* srci = w.idx[buf];
    float* dst = w.cols[buf ^ 1];
    int32_t* dsti = w.idx[buf ^ 1];
    const unsigned g_nw = (g_nn + kWavesPerBlock - 1) / kWavesPerBlock;
    if (nn_l <= w.split_block_nodes)  // few nodes: a workgroup each
        k_sample_block<<<g_nn, kSampleMax, 0, st>>>(cur, src, w.psamp, n, w.d, w.samples, w.dimv,
                                                    w.hist);
    else
        k_sample<<<g_nw, kBlock, 0, st>>>(cur, src, w.psamp, n, w.d, w.samples, w.dimv, w.hist);
    k_hist<<<g_nbh, kBlock, 0, st>>>(cur, w.dimv, w.samples, src, n, w.hist, w.crow);
    if (nn_l <= w.split_block_nodes)  // few large nodes: a block each
        k_choose<<<g_nn, kBlock, 0, st>>>(cur, w.dimv, w.samples, w.hist, w.crow, src, n, w.d,
                                          w.W, w.leaf, w.splitv, w.blk_off, w.nleft, w.planv);
    else
        k_choose_wave<<<g_nw, kBlock, 0, st>>>(cur, w.dimv, w.samples, w.hist, w.crow, src, n,
                                               w.d, w.W, w.leaf, w.splitv, w.blk_off, w.nleft,
                                               w.planv);
    k_plan_local<<<blocks_for(nn_l, kPlanBlock), kPlanBlock, 0, st>>>(cur, w.planv, w.planx,
                                                                       w.pblk, w.g);
    k_plan_top<<<1, kPlanBlock, 0, st>>>(cur, nxt, w.pblk, w.g, w.rng, level, w.big_cap,
                                         w.sub_cap, w.nn_cap, w.nb_cap, w.nbh_cap, w.ps_cap);
    // large-node levels (the partition's kLarge instance: pre-gathered samples,
    // the split column read once) while the largest tree's children can still
    // hold kPreSampleMin points (splits near the median halve the nodes)
    const bool pres = level < 62 && (w.largest >> (level + 1)) >= kPreSampleMin;
    k_plan_write<<<blocks_for(nn_l, kBlock), kBlock, 0, st>>>(
        cur, nxt, w.dimv, w.splitv, w.nleft, w.planx, w.pblk, w.leaf, w.W, w.max_depth, buf ^ 1,
        w.big, w.subs, w.cslot, pres ? 1 : 0, w.g);
    const int64_t nn_next = std::min<int64_t>(2 * nn_l, w.nn_cap);
    const int64_t fill = std::min<int64_t>(n / kChunk + nn_next + 1, w.nb_cap);
    k_plan_fill<<<blocks_for(fill, kBlock), kBlock, 0, st>>>(nxt);
    if (prof) prof_part_mark(st);
    (pres ? k_scatter<true> : k_scatter<false>)<<<g_nb, kBlock, 0, st>>>(
        cur, w.dimv, w.splitv, w.blk_off, w.nleft, w.cslot, w.ps_cap, src, srci, dst, dsti,
        w.psamp, n, w.d);
    if (prof) prof_part_mark(st);
}

}  // namespace

int32_t finish_max_points(int32_t) { return kWave * kGlobalRows; }

// Points of the LDS tile of a finish wavefront for subtrees of at most W
// points: the subtree nodes above it are split in registers from HBM.
int32_t finish_tile_points(int32_t d, int32_t w)
{
    return std::min(w, kWave * finish_rows(d));
}

size_t finish_lds_bytes_per_wave(int32_t d, int32_t w)
{
    // X [d][W] floats, indices [W] int32, permutation [W] u16, stack
    size_t b = (size_t)4 * d * w + (size_t)4 * w + (size_t)2 * w + sizeof(int4) * kStack;
    return (b + 15) & ~(size_t)15;
}

int32_t default_subtree_points(int32_t d) { return finish_max_points(d); }

// ---------------------------------------------------------------------------
// Device-side steps shared by the eager build and build plans: level 0 from
// one uploaded copy, the end of the level passes, the subtree id bases and
// the run status, so that no step between kernels needs the host.
// ---------------------------------------------------------------------------

// Blocks of the strided finish launch that takes the subtrees past the main
// grid of a plan run.
constexpr int kTailBlocks = 256;

// Status words of a build.
enum { PS_ERR = 0, PS_NSUB = 1, PS_NSUB_COMPACT = 2, PS_TOTAL = 3, PS_DEPTH = 4, PS_COUNT = 8 };

// Level 0 as uploaded (once per build, or once per plan): its node list; its
// block tables (nb0 partition blocks, nbh0 histogram blocks) are derived on
// the device from each node's first block.
struct PlanLevel0 {
    const int32_t* f;        // [8][nn0]: start, count, id, parent, depth, blk0, nblk, hblk0
    const SubEntry* small;   // [n_small]: roots that go straight to the subtree finish
    int32_t nn0, nb0, nbh0, n_small, T;
};

// The node whose first block (first[0 .. nn)) is the largest <= b.
__device__ inline int owner_of_block(const int32_t* __restrict__ first, int nn, int b)
{
    int lo = 0, hi = nn - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Start of a run: counters, status and the tree's query error count to zero.
__global__ void k_run_init(int32_t* __restrict__ g, int32_t* __restrict__ status,
                           int32_t* __restrict__ flags, unsigned long long* __restrict__ bad)
{
    const int t = threadIdx.x;
    if (t < G_COUNT) g[t] = 0;
    if (t < PS_COUNT) status[t] = 0;
    if (t < 2) flags[t] = 0;
    if (t == 0) *bad = 0;
}

// Level 0 from its uploaded copy; after the ingest, so that a non-finite
// coordinate empties the level and the subtree list (nothing is split).
__global__ void k_run_level0(PlanLevel0 P, Level L0, SubEntry* __restrict__ subs,
                             int32_t* __restrict__ g, int32_t* __restrict__ rng,
                             int32_t* __restrict__ status)
{
    const bool bad = g[G_NONFINITE] != 0;
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t* const dst[8] = {L0.start, L0.count, L0.id, L0.parent, L0.depth, L0.blk0, L0.nblk,
                             L0.hblk0};
    for (int64_t i = i0; i < 8 * (int64_t)P.nn0; i += stride)
        dst[i / P.nn0][i % P.nn0] = P.f[i];
    const int32_t* blk0 = P.f + 5 * (int64_t)P.nn0;
    const int32_t* hblk0 = P.f + 7 * (int64_t)P.nn0;
    for (int64_t i = i0; i < P.nb0; i += stride) {
        const int o = owner_of_block(blk0, P.nn0, (int)i);
        L0.bnode[i] = o;
        L0.bbeg[i] = ((int)i - blk0[o]) * kChunk;
    }
    for (int64_t i = i0; i < P.nbh0; i += stride) {
        const int o = owner_of_block(hblk0, P.nn0, (int)i);
        L0.hnode[i] = o;
        L0.hbeg[i] = ((int)i - hblk0[o]) * kHistChunk;
    }
    for (int64_t i = i0; i < P.n_small; i += stride) subs[i] = P.small[i];
    for (int64_t i = i0; i < P.nn0; i += stride) L0.sslot[i] = -1;  // roots gather their sample
    if (i0 == 0) {
        if (P.nn0) {
            L0.cnt[0] = bad ? 0 : P.nn0;
            L0.cnt[1] = bad ? 0 : P.nb0;
            L0.cnt[2] = bad ? 0 : P.nbh0;
        }
        g[G_NEXT_ID] = P.T;
        g[G_NSUB] = bad ? 0 : P.n_small;
        rng[0] = 0;
        rng[1] = bad ? 0 : P.T;
        if (bad) status[PS_ERR] = KNN_ENOTFINITE;
    }
}

// After the level passes: an error, or nodes left over once the planned
// passes ran out, stops the run; the subtree passes then see no subtrees and
// the box pass sees empty depth ranges.
__global__ void k_run_levels_done(const int32_t* __restrict__ left, const int32_t* __restrict__ g,
                                  int32_t* __restrict__ rng, int n_rng,
                                  int32_t* __restrict__ status)
{
    if (threadIdx.x != 0) return;
    int err = status[PS_ERR];
    if (!err && g[G_ERR]) err = g[G_ERR] == KNN_EDEPTH ? KNN_EDEPTH : KNN_EDEVICE;
    if (!err && left && *left != 0) err = KNN_EDEPTH;
    status[PS_ERR] = err;
    status[PS_NSUB] = err ? 0 : g[G_NSUB];
    if (err)
        for (int j = 0; j < 2 * n_rng; ++j) rng[j] = 0;
}

// Final ids of the subtree nodes: subtree i's nodes other than its root get
// ids base[i] .. base[i] + sub_nodes[i] - 2, after the level-pass ids, in
// subtree order (the eager build's host prefix sum).  One block, over passes
// of 8192 subtrees staged in LDS (coalesced loads and stores; each thread
// scans 8 consecutive subtrees).  A finish error (or too many nodes) stops
// the run as k_run_levels_done does.
__global__ __launch_bounds__(kPlanBlock) void k_run_bases(
    const int32_t* __restrict__ sub_nodes, const int32_t* __restrict__ g,
    const int32_t* __restrict__ flags, int32_t* __restrict__ base,
    int32_t* __restrict__ status, int64_t node_cap, int32_t* __restrict__ rng, int n_rng)
{
    constexpr int kChunkN = 8192;               // subtrees per pass, staged in LDS
    constexpr int kPer = kChunkN / kPlanBlock;  // consecutive subtrees per thread
    __shared__ int32_t tile[kChunkN];
    __shared__ long long wsum[kPlanBlock / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int ns = status[PS_NSUB];
    const int64_t n_big = g[G_NEXT_ID];
    long long carry = n_big;  // first id of the pass's first subtree's nodes
    for (int c0 = 0; c0 < ns; c0 += kChunkN) {
        const int cn = min(kChunkN, ns - c0);
        for (int i = t; i < cn; i += kPlanBlock) tile[i] = sub_nodes[c0 + i] - 1;
        __syncthreads();
        int v[kPer];
        long long mine = 0;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int i = t * kPer + r;
            v[r] = i < cn ? tile[i] : 0;
            mine += v[r];
        }
        long long x = mine;
        for (int o = 1; o < 64; o <<= 1) {
            const long long y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        long long before = 0, all = 0;
        for (int j = 0; j < kPlanBlock / 64; ++j) {
            if (j < w) before += wsum[j];
            all += wsum[j];
        }
        long long run = carry + before + x - mine;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int i = t * kPer + r;
            if (i < cn) tile[i] = (int32_t)run;
            run += v[r];
        }
        carry += all;
        __syncthreads();
        for (int i = t; i < cn; i += kPlanBlock) base[c0 + i] = tile[i];
        __syncthreads();  // tile and wsum are reused by the next pass
    }
    const long long all = carry - n_big;
    if (t == 0) {
        const long long total = n_big + all;
        int err = status[PS_ERR];
        if (!err && flags[0]) err = flags[0] == KNN_EDEPTH ? KNN_EDEPTH : KNN_EDEVICE;
        if (!err && total > node_cap) err = KNN_EDEVICE;
        status[PS_ERR] = err;
        status[PS_NSUB_COMPACT] = err ? 0 : ns;
        status[PS_TOTAL] = err ? 0 : (int32_t)total;
        status[PS_DEPTH] = flags[1];
        if (err)  // subtree roots stay unwritten: no box pass may read below them
            for (int j = 0; j < 2 * n_rng; ++j) rng[j] = 0;
    }
}

// End of a run.  After an error every root becomes a bucket holding only the
// pad row past the last point, whose index word is -1: the tree stays safe to
// query (results are padding-like rows), and knn_build_plan_finish reports the
// error.  Without an error that index word goes back to 0.
__global__ void k_run_done(const int32_t* __restrict__ status, NodeRec* __restrict__ nodes,
                           float* __restrict__ bbox, float* __restrict__ pts, int64_t n, int d,
                           int T)
{
    const bool err = status[PS_ERR] != 0;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) pts[n * (d + 1) + d] = __int_as_float(err ? -1 : 0);
    if (!err || i >= T) return;
    nodes[i] = NodeRec{(int32_t)n, -1, 0.0f, -1};
    for (int t = 0; t < 2 * d; ++t) bbox[(int64_t)i * 2 * d + t] = 0.0f;
}


// The words of level 0's upload: the node fields, then the small roots'
// subtree entries; and the device view of them at `dev`.
std::vector<int32_t> level0_words(const Level0Host& h0)
{
    std::vector<int32_t> w;
    for (int k = 0; k < 8; ++k) w.insert(w.end(), h0.f[k].begin(), h0.f[k].end());
    const size_t at = w.size();
    w.resize(at + h0.small.size() * (sizeof(SubEntry) / sizeof(int32_t)));
    if (!h0.small.empty()) std::memcpy(w.data() + at, h0.small.data(), sizeof(SubEntry) * h0.small.size());
    return w;
}

PlanLevel0 level0_view(const Level0Host& h0, const int32_t* dev, int32_t T)
{
    const size_t nn0 = h0.big_roots.size();
    return PlanLevel0{dev, reinterpret_cast<const SubEntry*>(dev + 8 * nn0), (int32_t)nn0,
                      h0.nb0, h0.nbh0, (int32_t)h0.small.size(), T};
}

unsigned level0_blocks(const PlanLevel0& l0)
{
    const int64_t items = std::max<int64_t>({8 * (int64_t)l0.nn0, l0.nb0, l0.nbh0, l0.n_small, 1});
    return (unsigned)std::min<int64_t>(blocks_for(items, kBlock), 4096);
}

// The error a build's status word records, as a return code with its message.
int status_error(int32_t code)
{
    switch (code) {
    case KNN_OK: return KNN_OK;
    case KNN_ENOTFINITE: return fail(KNN_ENOTFINITE, "an input coordinate is NaN or infinite");
    case KNN_EDEPTH: return fail(KNN_EDEPTH, "tree deeper than max_depth");
    default: return fail(KNN_EDEVICE, "the build overflowed its buffers");
    }
}

int build_tree(const float* points, int64_t n, int32_t d, int32_t leaf, int32_t max_depth,
               int32_t W, int64_t split_block_nodes, const int64_t* offsets, int32_t T,
               hipStream_t st, knn_tree** out)
{
    FinishFn ff = finish_for(d);
    if (!ff) return fail(KNN_EINVAL, "unsupported dimension");
    prof_mark(st, 0);
    prof_part_begin();
    // level 0's host words outlive every buffer below, whose release waits
    // for the stream (and so for their upload)
    const Level0Host h0 = level0_tables(offsets, T, W, leaf);
    const std::vector<int32_t> l0host = level0_words(h0);
    const int64_t nd = n * d;
    // scratch and the tree's own buffers (pts, nodes, bbox) come from the
    // library's block cache: a build that follows another, or a freed tree,
    // reuses that memory instead of mapping fresh pages while the device waits
    DevBuf colsA(st), colsB(st), idxA(st), idxB(st), pts(st), gbuf(st), l0buf(st);
    // padded by one finish tile of rows: the finish reads whole rows of 64
    // points, up to 64 * kGlobalRows - 1 elements past a node's last point
    const int64_t tail = (int64_t)kWave * kGlobalRows;
    KNN_HIP(colsA.alloc(sizeof(float) * (nd + tail)));
    KNN_HIP(colsB.alloc(sizeof(float) * (nd + tail)));
    KNN_HIP(idxA.alloc(sizeof(int32_t) * (n + tail)));
    KNN_HIP(idxB.alloc(sizeof(int32_t) * (n + tail)));
    KNN_HIP(pts.alloc(sizeof(float) * (n + kRowPad) * (d + 1)));
    KNN_HIP(hipMemsetAsync(pts.as<float>() + n * (d + 1), 0, sizeof(float) * kRowPad * (d + 1), st));
    // build counters, status words and the finish's error and depth flags
    constexpr int kWords = G_COUNT + PS_COUNT + 2;
    KNN_HIP(gbuf.alloc(sizeof(int32_t) * kWords));
    int32_t* g = gbuf.as<int32_t>();
    int32_t* status = g + G_COUNT;
    int32_t* flags = status + PS_COUNT;
    KNN_HIP(hipMemsetAsync(g, 0, sizeof(int32_t) * kWords, st));
    KNN_HIP(l0buf.alloc(sizeof(int32_t) * l0host.size()));
    KNN_HIP(hipMemcpyAsync(l0buf.p, l0host.data(), sizeof(int32_t) * l0host.size(),
                           hipMemcpyHostToDevice, st));
    {
        const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 65536);
        k_ingest<<<(unsigned)blocks, kBlock, 0, st>>>(points, n, d, colsA.as<float>(),
                                                      idxA.as<int32_t>(), g);
        KNN_HIP(hipGetLastError());
    }
    prof_mark(st, 1);

    // ---- level passes: nodes above W points (and above the bucket size) -------
    // a level's nodes hold more than W points each and are disjoint
    const int64_t nn_cap = n / (W + 1) + 1;
    const int64_t nb_cap = n / kChunk + nn_cap + 1;
    const int64_t nbh_cap = n / kHistChunk + nn_cap + 1;
    // a level's children with pre-gathered samples hold kPreSampleMin points each
    const int64_t ps_cap = n / kPreSampleMin + 1;
    const int64_t lv_cap = (int64_t)max_depth + 2;
    // every level-pass node and subtree entry descends from a level node
    const int64_t big_cap = T + 2 * nn_cap * lv_cap + 2;
    const int64_t sub_cap = std::min<int64_t>(n, big_cap);
    const std::vector<int32_t>& big_roots = h0.big_roots;
    const int32_t nn0 = (int32_t)big_roots.size();
    LevelMem lvA(st), lvB(st);
    DevBuf dimv(st), splitv(st), nleft(st), samples(st), hist(st), crow(st), psamp(st), cslot(st),
        blk_off(st),
        d_big(st), d_subs(st), d_rng(st), planv(st), planx(st), pblk(st);
    int32_t n_sub = (int32_t)h0.small.size(), n_big = T, n_levels = 1;
    std::vector<int32_t> h_g(G_COUNT + PS_COUNT, 0);
    if (nn0) {
        KNN_HIP(lvA.alloc(nn_cap, nb_cap, nbh_cap));
        KNN_HIP(lvB.alloc(nn_cap, nb_cap, nbh_cap));
        KNN_HIP(dimv.alloc(sizeof(int32_t) * nn_cap));
        KNN_HIP(splitv.alloc(sizeof(float) * nn_cap));
        KNN_HIP(nleft.alloc(sizeof(int32_t) * nn_cap));
        KNN_HIP(samples.alloc(sizeof(float) * kWinStride * nn_cap));
        KNN_HIP(hist.alloc(sizeof(uint32_t) * kWinRow * nn_cap));
        KNN_HIP(crow.alloc(sizeof(uint16_t) * kCrowStride * nb_cap));
        KNN_HIP(psamp.alloc(sizeof(float) * kSampleMax * d * ps_cap));
        KNN_HIP(cslot.alloc(sizeof(int32_t) * 2 * nn_cap));
        KNN_HIP(blk_off.alloc(sizeof(uint32_t) * nb_cap));
        KNN_HIP(planv.alloc(sizeof(int32_t) * kPlanStride * nn_cap));
        KNN_HIP(planx.alloc(sizeof(int32_t) * kPlanStride * nn_cap));
        KNN_HIP(pblk.alloc(sizeof(int32_t) * kPlanStride * ((nn_cap + kPlanBlock - 1) / kPlanBlock)));
        KNN_HIP(d_big.alloc(sizeof(NodeRec) * big_cap));
        KNN_HIP(d_subs.alloc(sizeof(SubEntry) * sub_cap));
        KNN_HIP(d_rng.alloc(sizeof(int32_t) * 2 * (lv_cap + 1)));
    } else {
        KNN_HIP(d_big.alloc(sizeof(NodeRec) * T));
        KNN_HIP(d_subs.alloc(sizeof(SubEntry) * h0.small.size()));
        KNN_HIP(d_rng.alloc(sizeof(int32_t) * 2));
    }
    {   // level 0 and the small roots from the upload; a non-finite
        // coordinate leaves both empty (checked at the next host wait)
        const PlanLevel0 l0 = level0_view(h0, l0buf.as<int32_t>(), T);
        k_run_level0<<<level0_blocks(l0), kBlock, 0, st>>>(l0, lvA.L, d_subs.as<SubEntry>(), g,
                                                           d_rng.as<int32_t>(), status);
        KNN_HIP(hipGetLastError());
    }
    if (nn0) {
        // levels expected for balanced splits; the host checks for more after that
        const int expected = expected_levels(h0.largest, W, leaf);
        LevelWork lw{};
        lw.cols[0] = colsA.as<float>();
        lw.cols[1] = colsB.as<float>();
        lw.idx[0] = idxA.as<int32_t>();
        lw.idx[1] = idxB.as<int32_t>();
        lw.dimv = dimv.as<int32_t>();
        lw.splitv = splitv.as<float>();
        lw.nleft = nleft.as<int32_t>();
        lw.samples = samples.as<float>();
        lw.hist = hist.as<uint32_t>();
        lw.crow = crow.as<uint16_t>();
        lw.psamp = psamp.as<float>();
        lw.cslot = cslot.as<int32_t>();
        lw.blk_off = blk_off.as<uint32_t>();
        lw.planv = planv.as<int32_t>();
        lw.planx = planx.as<int32_t>();
        lw.pblk = pblk.as<int32_t>();
        lw.big = d_big.as<NodeRec>();
        lw.subs = d_subs.as<SubEntry>();
        lw.rng = d_rng.as<int32_t>();
        lw.g = g;
        lw.n = n;
        lw.d = d;
        lw.leaf = leaf;
        lw.W = W;
        lw.max_depth = max_depth;
        lw.split_block_nodes = split_block_nodes;
        lw.nn0 = nn0;
        lw.largest = h0.largest;
        lw.nn_cap = nn_cap;
        lw.nb_cap = nb_cap;
        lw.nbh_cap = nbh_cap;
        lw.big_cap = big_cap;
        lw.sub_cap = sub_cap;
        lw.ps_cap = ps_cap;
        Level cur = lvA.L, nxt = lvB.L;
        int buf = 0;
        for (int level = 0;; ++level) {
            if (level >= lv_cap) return fail(KNN_EDEPTH, "tree deeper than max_depth");
            enqueue_level(lw, cur, nxt, level, buf, true, st);
            KNN_HIP(hipGetLastError());
            n_levels = level + 2;  // depth ranges 0 .. level + 1 are recorded
            std::swap(cur, nxt);
            buf ^= 1;
            if (level + 1 >= expected) {
                // the counters and the status words in one read
                KNN_HIP(hipMemcpyAsync(h_g.data(), g, sizeof(int32_t) * (G_COUNT + PS_COUNT),
                                       hipMemcpyDeviceToHost, st));
                KNN_HIP(hipStreamSynchronize(st));
                if (h_g[G_COUNT + PS_ERR]) return status_error(h_g[G_COUNT + PS_ERR]);
                if (h_g[G_ERR] == KNN_EDEPTH) return fail(KNN_EDEPTH, "tree deeper than max_depth");
                if (h_g[G_ERR]) return fail(KNN_EDEVICE, "level bookkeeping overflowed its buffers");
                if (h_g[G_LEVEL_NODES] == 0) break;
            }
        }
        n_sub = h_g[G_NSUB];
        n_big = h_g[G_NEXT_ID];
        {
            uint64_t moved = 0;
            std::memcpy(&moved, &h_g[G_MOVED], sizeof(moved));
            prof_part_points((double)moved);
        }
        lvA.mem.reset(); lvB.mem.reset(); samples.reset(); hist.reset(); crow.reset();
        psamp.reset(); cslot.reset();
        blk_off.reset(); dimv.reset(); splitv.reset(); nleft.reset(); planv.reset(); planx.reset();
        pblk.reset();
    }
    // the subtree count on the device (0 after a non-finite coordinate)
    k_run_levels_done<<<1, kWave, 0, st>>>(nullptr, g, d_rng.as<int32_t>(), n_levels, status);
    prof_mark(st, 2);

    // ---- subtree finish -----------------------------------------------------
    DevBuf tnodes(st), tbox(st), subn(st), d_base(st);
    KNN_HIP(tnodes.alloc(sizeof(NodeRec) * 2 * n));
    KNN_HIP(tbox.alloc(sizeof(float) * 2 * n * 2 * d));
    KNN_HIP(subn.alloc(sizeof(int32_t) * n_sub));
    KNN_HIP(d_base.alloc(sizeof(int32_t) * n_sub));
    const int32_t Wt = finish_tile_points(d, W);
    const size_t per_wave = finish_lds_bytes_per_wave(d, Wt);
    const size_t lds = per_wave * kWavesPerBlock;
    const int32_t fblocks = (n_sub + kWavesPerBlock - 1) / kWavesPerBlock;
    if (lds > 64 * 1024)
        KNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(ff),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(ff, dim3(fblocks), dim3(kBlock), lds, st, d_subs.as<SubEntry>(), 0, n_sub,
                       status + PS_NSUB, colsA.as<float>(), idxA.as<int32_t>(), colsB.as<float>(),
                       idxB.as<int32_t>(), n, leaf, Wt, max_depth, per_wave, pts.as<float>(),
                       tnodes.as<NodeRec>(), tbox.as<float>(), subn.as<int32_t>(), flags,
                       flags + 1);
    KNN_HIP(hipGetLastError());
    // ids: level-pass nodes first, then each subtree's nodes in subtree order
    k_run_bases<<<1, kPlanBlock, 0, st>>>(subn.as<int32_t>(), g, flags, d_base.as<int32_t>(),
                                          status, (int64_t)INT32_MAX, d_rng.as<int32_t>(),
                                          n_levels);
    KNN_HIP(hipGetLastError());
    int32_t h_status[PS_COUNT] = {};
    KNN_HIP(hipMemcpyAsync(h_status, status, sizeof(h_status), hipMemcpyDeviceToHost, st));
    KNN_HIP(hipStreamSynchronize(st));
    prof_mark(st, 3);
    if (int rc = status_error(h_status[PS_ERR])) return rc;

    // ---- records and boxes ----------------------------------------------------
    const int64_t total = h_status[PS_TOTAL];
    DevBuf nodes(st), bbox(st), badc(st);
    KNN_HIP(nodes.alloc(sizeof(NodeRec) * total));
    KNN_HIP(bbox.alloc(sizeof(float) * total * 2 * d));
    KNN_HIP(badc.alloc(sizeof(unsigned long long)));
    KNN_HIP(hipMemsetAsync(badc.p, 0, sizeof(unsigned long long), st));
    if (n_big > 1)
        KNN_HIP(hipMemcpyAsync(nodes.p, d_big.p, sizeof(NodeRec) * n_big, hipMemcpyDeviceToDevice, st));
    k_compact<<<fblocks, kBlock, 0, st>>>(d_subs.as<SubEntry>(), n_sub, status + PS_NSUB_COMPACT,
                                          subn.as<int32_t>(), d_base.as<int32_t>(),
                                          tnodes.as<NodeRec>(), tbox.as<float>(), d,
                                          nodes.as<NodeRec>(), bbox.as<float>());
    KNN_HIP(hipGetLastError());
    for (int dep = n_levels - 1; dep >= 0; --dep) {
        const int64_t cap = std::min<int64_t>(dep < 40 ? (int64_t)T << dep : total, total);
        k_bbox_up<<<blocks_for(cap, kBlock), kBlock, 0, st>>>(d_rng.as<int32_t>() + 2 * dep,
                                                             nodes.as<NodeRec>(), bbox.as<float>(), d);
        KNN_HIP(hipGetLastError());
    }
    KNN_HIP(hipStreamSynchronize(st));
    prof_mark(st, 4);

    knn_tree* t = new knn_tree();
    t->n = n;
    t->d = d;
    t->leaf = leaf;
    t->n_trees = T;
    t->depth = h_status[PS_DEPTH];
    t->sub_pts = W;
    t->n_nodes = total;
    (void)hipGetDevice(&t->device);
    t->bytes = (int64_t)(pts.bytes + nodes.bytes + bbox.bytes + badc.bytes);
    t->pts = pts.as<float>();
    t->nodes = nodes.as<NodeRec>();
    t->bbox = bbox.as<float>();
    t->bad = badc.as<unsigned long long>();
    pts.release();
    nodes.release();
    bbox.release();
    badc.release();
    *out = t;
    return KNN_OK;
}

}  // namespace knn

// ---------------------------------------------------------------------------
// Build plans: the build above for a fixed point count and forest layout,
// with every buffer sized once at creation and no host round trip between
// kernels.  A run is a fixed sequence of kernel launches (no allocation,
// copy, fill or wait), so a HIP graph can capture it; results come back
// through device status words that knn_build_plan_finish reads.
// ---------------------------------------------------------------------------

struct knn_build_plan {
    int32_t device = 0;
    int64_t n = 0;
    int32_t d = 0, leaf = 0, W = 0, max_depth = 0, T = 0, levels = 0;
    int64_t split_block_nodes = 0;
    int64_t nn_cap = 0, nb_cap = 0, nbh_cap = 0, big_cap = 0, sub_cap = 0, node_cap = 0, ps_cap = 0;
    int32_t Wt = 0;
    size_t per_wave = 0, lds = 0;
    unsigned fgrid = 0;
    knn::FinishFn ff = nullptr;       // one subtree per wavefront
    knn::FinishFn ff_tail = nullptr;  // strided, for subtrees past ff's grid
    std::vector<void*> blocks;  // every device block the plan holds (block cache)
    knn::LevelWork lw{};
    knn::Level lv[2]{};
    knn::PlanLevel0 l0{};
    float* pts = nullptr;
    knn::NodeRec* tnodes = nullptr;
    float* tbox = nullptr;
    int32_t* subn = nullptr;
    int32_t* flags = nullptr;
    int32_t* base = nullptr;
    int32_t* status = nullptr;
    knn::NodeRec* nodes = nullptr;
    float* bbox = nullptr;
    knn_tree* tree = nullptr;
    hipEvent_t last = nullptr;  // recorded after the latest run enqueued outside a capture
    bool ran = false;
};

namespace knn {

namespace {

template <class T>
hipError_t plan_alloc(knn_build_plan* P, T** p, size_t count)
{
    void* q = nullptr;
    const hipError_t e = cache_alloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    P->blocks.push_back(q);
    *p = static_cast<T*>(q);
    return hipSuccess;
}

void plan_release(knn_build_plan* P)
{
    for (void* q : P->blocks) cache_free(q);
    P->blocks.clear();
    if (P->last) (void)hipEventDestroy(P->last);
    delete P->tree;
    delete P;
}

}  // namespace

int plan_create(int64_t n, int32_t d, const int64_t* offsets, int32_t T, int32_t leaf,
                int32_t max_depth, int32_t W, int64_t split_block_nodes, hipStream_t st,
                knn_build_plan** out)
{
    FinishFn ff = finish_for(d);
    if (!ff) return fail(KNN_EINVAL, "unsupported dimension");
    const Level0Host h0 = level0_tables(offsets, T, W, leaf);
    int64_t biggest = 0;
    for (int32_t r = 0; r < T; ++r) biggest = std::max(biggest, offsets[r + 1] - offsets[r]);
    if (max_depth == 0) {  // balanced depth of the largest tree, with room for uneven splits
        int dep = 0;
        for (int64_t c = biggest; c > leaf; c = (c + 1) / 2) ++dep;
        max_depth = dep + 8;
    }
    std::unique_ptr<knn_build_plan, void (*)(knn_build_plan*)> P(new knn_build_plan(),
                                                                  plan_release);
    (void)hipGetDevice(&P->device);
    P->n = n;
    P->d = d;
    P->leaf = leaf;
    P->W = W;
    P->max_depth = max_depth;
    P->T = T;
    P->split_block_nodes = split_block_nodes;
    const int nn0 = (int)h0.big_roots.size();
    P->levels = nn0 ? std::min(expected_levels(h0.largest, W, leaf) + 4, max_depth + 1) : 0;
    // capacities as in the eager build, with the planned passes as the depth
    const int64_t lv_cap = (int64_t)P->levels + 1;
    P->nn_cap = n / (W + 1) + 1;
    P->nb_cap = n / kChunk + P->nn_cap + 1;
    P->nbh_cap = n / kHistChunk + P->nn_cap + 1;
    P->ps_cap = n / kPreSampleMin + 1;
    P->big_cap = T + 2 * P->nn_cap * lv_cap + 2;
    P->sub_cap = std::min<int64_t>(n, P->big_cap);
    P->node_cap = std::max<int64_t>(2 * n + T, P->big_cap);
    if (P->node_cap > INT32_MAX) return fail(KNN_EINVAL, "too many nodes for int32 ids");
    const int64_t nd = n * d, tail = (int64_t)kWave * kGlobalRows;
    LevelWork& w = P->lw;
    int32_t* g = nullptr;
    int32_t* lvbuf[2] = {nullptr, nullptr};
    int32_t* rng = nullptr;
    int32_t* l0buf = nullptr;
    KNN_HIP(plan_alloc(P.get(), &w.cols[0], nd + tail));
    KNN_HIP(plan_alloc(P.get(), &w.cols[1], nd + tail));
    KNN_HIP(plan_alloc(P.get(), &w.idx[0], n + tail));
    KNN_HIP(plan_alloc(P.get(), &w.idx[1], n + tail));
    KNN_HIP(plan_alloc(P.get(), &P->pts, (n + kRowPad) * (d + 1)));
    KNN_HIP(plan_alloc(P.get(), &g, G_COUNT));
    KNN_HIP(plan_alloc(P.get(), &rng, 2 * (lv_cap + 1)));
    KNN_HIP(plan_alloc(P.get(), &w.subs, P->sub_cap));
    KNN_HIP(plan_alloc(P.get(), &P->tnodes, 2 * n));
    KNN_HIP(plan_alloc(P.get(), &P->tbox, 2 * n * 2 * d));
    KNN_HIP(plan_alloc(P.get(), &P->subn, P->sub_cap));
    KNN_HIP(plan_alloc(P.get(), &P->base, P->sub_cap));
    KNN_HIP(plan_alloc(P.get(), &P->flags, 2));
    KNN_HIP(plan_alloc(P.get(), &P->status, PS_COUNT));
    KNN_HIP(plan_alloc(P.get(), &P->nodes, P->node_cap));
    KNN_HIP(plan_alloc(P.get(), &P->bbox, P->node_cap * 2 * d));
    unsigned long long* bad = nullptr;
    KNN_HIP(plan_alloc(P.get(), &bad, 1));
    if (nn0) {
        for (int k = 0; k < 2; ++k) {
            KNN_HIP(plan_alloc(P.get(), &lvbuf[k], level_words(P->nn_cap, P->nb_cap, P->nbh_cap)));
            P->lv[k] = carve_level(lvbuf[k], P->nn_cap, P->nb_cap, P->nbh_cap);
        }
        KNN_HIP(plan_alloc(P.get(), &w.dimv, P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.splitv, P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.nleft, P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.samples, (size_t)kWinStride * P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.hist, (size_t)kWinRow * P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.crow, (size_t)kCrowStride * P->nb_cap));
        KNN_HIP(plan_alloc(P.get(), &w.psamp, (size_t)kSampleMax * d * P->ps_cap));
        KNN_HIP(plan_alloc(P.get(), &w.cslot, 2 * P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.blk_off, P->nb_cap));
        KNN_HIP(plan_alloc(P.get(), &w.planv, (size_t)kPlanStride * P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.planx, (size_t)kPlanStride * P->nn_cap));
        KNN_HIP(plan_alloc(P.get(), &w.pblk,
                           (size_t)kPlanStride * ((P->nn_cap + kPlanBlock - 1) / kPlanBlock)));
    }
    // level 0 and the small roots, uploaded once
    {
        const std::vector<int32_t> host = level0_words(h0);
        KNN_HIP(plan_alloc(P.get(), &l0buf, host.size()));
        if (!host.empty())
            KNN_HIP(hipMemcpyAsync(l0buf, host.data(), sizeof(int32_t) * host.size(),
                                   hipMemcpyHostToDevice, st));
        // the pad rows past the last point read as zeros
        KNN_HIP(hipMemsetAsync(P->pts + n * (d + 1), 0, sizeof(float) * kRowPad * (d + 1), st));
        KNN_HIP(hipStreamSynchronize(st));  // the host copy dies here
    }
    P->l0 = level0_view(h0, l0buf, T);
    w.big = P->nodes;  // level-pass records go straight to their final ids
    w.rng = rng;
    w.g = g;
    w.n = n;
    w.d = d;
    w.leaf = leaf;
    w.W = W;
    w.max_depth = max_depth;
    w.split_block_nodes = split_block_nodes;
    w.nn0 = nn0;
    w.largest = h0.largest;
    w.nn_cap = P->nn_cap;
    w.nb_cap = P->nb_cap;
    w.nbh_cap = P->nbh_cap;
    w.big_cap = P->big_cap;
    w.sub_cap = P->sub_cap;
    w.ps_cap = P->ps_cap;
    P->ff = ff;
    P->ff_tail = finish_for(d, true);
    P->Wt = finish_tile_points(d, W);
    P->per_wave = finish_lds_bytes_per_wave(d, P->Wt);
    P->lds = P->per_wave * kWavesPerBlock;
    if (P->lds > 64 * 1024)
        for (FinishFn f : {P->ff, P->ff_tail})
            KNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)P->lds));
    // one wavefront per subtree for the usual count (subtrees hold more than
    // W / 2 points when splits are near even); more are taken in strides
    const int64_t usual = std::min<int64_t>(P->sub_cap, 3 * n / W + 2 * (int64_t)T + 256);
    P->fgrid = (unsigned)((usual + kWavesPerBlock - 1) / kWavesPerBlock);

    knn_tree* t = new knn_tree();
    t->n = n;
    t->d = d;
    t->leaf = leaf;
    t->n_trees = T;
    t->depth = max_depth;  // a bound that holds for every successful run
    t->sub_pts = W;
    t->n_nodes = 0;
    t->device = P->device;
    t->bytes = (int64_t)(sizeof(float) * (n + kRowPad) * (d + 1) +
                         (sizeof(NodeRec) + sizeof(float) * 2 * d) * P->node_cap);
    t->pts = P->pts;
    t->nodes = P->nodes;
    t->bbox = P->bbox;
    t->bad = bad;
    t->plan_owned = true;
    P->tree = t;
    KNN_HIP(hipEventCreateWithFlags(&P->last, hipEventDisableTiming));
    *out = P.release();
    return KNN_OK;
}

int plan_run(knn_build_plan* P, const float* points, hipStream_t st)
{
    const int64_t n = P->n;
    const int d = P->d, T = P->T;
    const LevelWork& w = P->lw;
    k_run_init<<<1, 64, 0, st>>>(w.g, P->status, P->flags, P->tree->bad);
    {
        const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 65536);
        k_ingest<<<(unsigned)blocks, kBlock, 0, st>>>(points, n, d, w.cols[0], w.idx[0], w.g);
    }
    k_run_level0<<<level0_blocks(P->l0), kBlock, 0, st>>>(P->l0, P->lv[0], w.subs, w.g, w.rng,
                                                          P->status);
    int buf = 0;
    for (int level = 0; level < P->levels; ++level) {
        enqueue_level(w, P->lv[buf], P->lv[buf ^ 1], level, buf, false, st);
        buf ^= 1;
    }
    k_run_levels_done<<<1, 64, 0, st>>>(P->levels ? P->lv[buf].cnt : nullptr, w.g, w.rng,
                                        P->levels + 1, P->status);
    hipLaunchKernelGGL(P->ff, dim3(P->fgrid), dim3(kBlock), P->lds, st, w.subs, 0, 0,
                       P->status + PS_NSUB, w.cols[0], w.idx[0], w.cols[1], w.idx[1], n, P->leaf,
                       P->Wt, P->max_depth, P->per_wave, P->pts, P->tnodes, P->tbox, P->subn,
                       P->flags, P->flags + 1);
    // subtrees past the main grid (uneven splits), if any
    hipLaunchKernelGGL(P->ff_tail, dim3(kTailBlocks), dim3(kBlock), P->lds, st, w.subs,
                       (int32_t)(P->fgrid * kWavesPerBlock), 0, P->status + PS_NSUB, w.cols[0],
                       w.idx[0], w.cols[1], w.idx[1], n, P->leaf, P->Wt, P->max_depth,
                       P->per_wave, P->pts, P->tnodes, P->tbox, P->subn, P->flags, P->flags + 1);
    k_run_bases<<<1, kPlanBlock, 0, st>>>(P->subn, w.g, P->flags, P->base, P->status,
                                          P->node_cap, w.rng, P->levels + 1);
    k_compact<<<P->fgrid, kBlock, 0, st>>>(w.subs, 0, P->status + PS_NSUB_COMPACT, P->subn,
                                           P->base, P->tnodes, P->tbox, d, P->nodes, P->bbox);
    for (int dep = P->levels; dep >= 0; --dep) {
        const int64_t cap = std::min<int64_t>(dep < 40 ? (int64_t)T << dep : P->node_cap,
                                              P->node_cap);
        k_bbox_up<<<blocks_for(cap, kBlock), kBlock, 0, st>>>(w.rng + 2 * dep, P->nodes, P->bbox,
                                                             d);
    }
    k_run_done<<<blocks_for(T, kBlock), kBlock, 0, st>>>(P->status, P->nodes, P->bbox, P->pts, n,
                                                          d, T);
    KNN_HIP(hipGetLastError());
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    KNN_HIP(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone) KNN_HIP(hipEventRecord(P->last, st));
    P->ran = true;
    return KNN_OK;
}

int plan_finish(knn_build_plan* P, hipStream_t st)
{
    if (!P->ran) return fail(KNN_EINVAL, "the plan has not run");
    int32_t h[PS_COUNT] = {};
    KNN_HIP(hipMemcpyAsync(h, P->status, sizeof(h), hipMemcpyDeviceToHost, st));
    KNN_HIP(hipStreamSynchronize(st));
    knn_tree* t = P->tree;
    t->n_nodes = h[PS_ERR] ? P->T : h[PS_TOTAL];
    return status_error(h[PS_ERR]);
}

int plan_destroy(knn_build_plan* P)
{
    int rc = KNN_OK;
    {   // queries on the plan's tree, then the latest run outside a capture
        std::lock_guard<std::mutex> lk(P->tree->use_mu);
        for (auto& u : P->tree->uses) {
            hipError_t e = hipEventSynchronize(u.second);
            if (e != hipSuccess && rc == KNN_OK) rc = hip_fail(e, "hipEventSynchronize");
            (void)hipEventDestroy(u.second);
        }
        P->tree->uses.clear();
    }
    if (P->ran) {
        hipError_t e = hipEventSynchronize(P->last);
        if (e != hipSuccess && rc == KNN_OK) rc = hip_fail(e, "hipEventSynchronize");
    }
    plan_release(P);
    return rc;
}

knn_tree* plan_tree(knn_build_plan* P) { return P->tree; }
int32_t plan_device(const knn_build_plan* P) { return P->device; }

}  // namespace knn
