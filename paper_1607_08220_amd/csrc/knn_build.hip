// kd-tree construction on gfx950 (Section III-A of arXiv 1607.08220).
//
// The paper builds the local tree breadth-first with all threads on the top
// levels (III-A ii), then lets each thread finish a subtree depth-first
// (III-A iii), then packs buckets (III-A iv).  Here:
//   * ingest:    caller AoS [n,d] -> SoA columns + index column
//   * level pass (nodes above `W` points), one node list per level:
//       k_sample   sample of min(1024, cnt) points, FP64 variance per dim,
//                  split dim = argmax, sorted sample of that dim (LDS bitonic)
//       k_hist     histogram of every node point over the sorted sample
//                  (per-lane binary search in LDS, LDS atomics)
//       k_choose   running counts C_j, j* = argmin |2 C_j - cnt|
//       k_count    per-wavefront count of points going left (ballot)
//       k_blkscan  per-node exclusive scan of block counts
//       k_scatter  stable partition of coordinates + index into the other
//                  ping-pong buffer (ballot + mbcnt ranks)
//   * k_finish:  one wavefront per node of at most W points builds its whole
//                subtree in LDS (every point is a sample there, so the split
//                is the exact value the histogram rule selects), computes the
//                tight boxes and writes the packed bucket rows
//   * k_compact: gives every subtree node its final id; k_bbox_up fills the
//                boxes of the level-pass nodes bottom-up.
// Node ids are deterministic: level-pass nodes in breadth-first order, then
// each subtree's nodes in the order the subtree list is kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "knn_internal.h"

namespace knn {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;       // 4
constexpr int kItems = 16;                           // elements per lane per block pass
constexpr int kWaveChunk = kWave * kItems;           // 1024 elements per wavefront
constexpr int kChunk = kBlock * kItems;              // 4096 elements per block
constexpr int kBins = kSampleMax + 1;                // histogram bins per node
constexpr int kStack = 32;                           // subtree DFS stack (entries)

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

// Pairwise FP64 sum over a[0..1023] (zero padded), a[i] += a[i + w] for
// w = 512 .. 1.  Thread t of the block holds a[t + 256 r], r = 0..3.
// Zero padding past the sample size leaves the sum equal to the same tree
// over the next power of two above the sample size.
__device__ double block_psum(const double a[4], double* red)
{
    const int t = threadIdx.x;
    double x0 = a[0] + a[2];  // w = 512
    double x1 = a[1] + a[3];
    red[t] = x0 + x1;         // w = 256
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) red[t] = red[t] + red[t + w];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// The same tree inside one wavefront: lane l holds a[l + 64 r], r = 0..15.
__device__ double wave_psum(double a[16])
{
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = a[r] + a[r + 8];  // w = 512
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = a[r] + a[r + 4];  // w = 256
#pragma unroll
    for (int r = 0; r < 2; ++r) a[r] = a[r] + a[r + 2];  // w = 128
    double v = a[0] + a[1];                              // w = 64
    for (int w = 32; w >= 1; w >>= 1) v = v + __shfl_down(v, w);
    return __shfl(v, 0);
}

// ---------------------------------------------------------------------------
// B0: ingest
// ---------------------------------------------------------------------------
__global__ void k_ingest(const float* __restrict__ aos, int64_t n, int d,
                         float* __restrict__ cols, int32_t* __restrict__ idx)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int t = 0; t < d; ++t) cols[(int64_t)t * n + i] = aos[i * d + t];
        idx[i] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------
// B1-B3: sample, split dimension, sorted sample (one block per node)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_sample(const int32_t* __restrict__ lv_start,
                                                   const int32_t* __restrict__ lv_count,
                                                   const float* __restrict__ cols, int64_t n,
                                                   int d, float* __restrict__ samples,
                                                   int32_t* __restrict__ out_dim)
{
    __shared__ double red[kBlock];
    __shared__ float sv[kSampleMax];
    const int node = blockIdx.x, t = threadIdx.x;
    const int64_t start = lv_start[node], c = lv_count[node];
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    double bestV = -1.0;
    int best = 0;
    for (int dd = 0; dd < d; ++dd) {
        const float* col = cols + (int64_t)dd * n + start;
        double a[4], q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int i = t + kBlock * r;
            a[r] = i < s ? (double)col[sample_pos(i, c, s)] : 0.0;
        }
        const double S = block_psum(a, red);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int i = t + kBlock * r;
            double w = (double)s * a[r] - S;
            q[r] = i < s ? w * w : 0.0;
        }
        const double V = block_psum(q, red);
        if (V > bestV) {
            bestV = V;
            best = dd;
        }
    }
    if (!(bestV > 0.0)) {  // sample constant in every dimension
        if (t == 0) out_dim[node] = -1;
        return;
    }
    const float* col = cols + (int64_t)best * n + start;
    int P = 1;
    while (P < s) P <<= 1;
    for (int i = t; i < P; i += kBlock) sv[i] = i < s ? col[sample_pos(i, c, s)] : INFINITY;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = t; i < P; i += kBlock) {
                int ixj = i ^ j;
                if (ixj > i) {
                    float x = sv[i], y = sv[ixj];
                    bool asc = (i & k) == 0;
                    if ((x > y) == asc) {
                        sv[i] = y;
                        sv[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = t; i < s; i += kBlock) samples[(int64_t)node * kSampleMax + i] = sv[i];
    if (t == 0) out_dim[node] = best;
}

// ---------------------------------------------------------------------------
// B4: histogram over the sorted sample (blocks over node chunks)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_hist(const int32_t* __restrict__ blk_node,
                                                 const int32_t* __restrict__ blk_begin,
                                                 const int32_t* __restrict__ lv_start,
                                                 const int32_t* __restrict__ lv_count,
                                                 const int32_t* __restrict__ dimv,
                                                 const float* __restrict__ samples,
                                                 const float* __restrict__ cols, int64_t n,
                                                 uint32_t* __restrict__ hist)
{
    __shared__ float sv[kSampleMax];
    __shared__ uint32_t h[kBins];
    const int b = blockIdx.x, t = threadIdx.x;
    const int node = blk_node[b];
    const int dim = dimv[node];
    if (dim < 0) return;
    const int64_t start = lv_start[node], c = lv_count[node];
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    const int64_t beg = blk_begin[b];
    const int64_t end = beg + kChunk < c ? beg + kChunk : c;
    for (int i = t; i < s; i += kBlock) sv[i] = samples[(int64_t)node * kSampleMax + i];
    for (int i = t; i <= s; i += kBlock) h[i] = 0u;
    __syncthreads();
    const float* col = cols + (int64_t)dim * n + start;
    for (int64_t e = beg + t; e < end; e += kBlock) {
        const float x = col[e];
        int pos = 0;  // number of sample values <= x
        for (int step = kSampleMax; step > 0; step >>= 1) {
            int np = pos + step;
            if (np <= s && sv[np - 1] <= x) pos = np;
        }
        atomicAdd(&h[pos], 1u);
    }
    __syncthreads();
    for (int i = t; i <= s; i += kBlock)
        if (h[i]) atomicAdd(&hist[(int64_t)node * kBins + i], h[i]);
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

__global__ __launch_bounds__(kBlock) void k_choose(const int32_t* __restrict__ lv_start,
                                                   const int32_t* __restrict__ lv_count,
                                                   int32_t* __restrict__ dimv,
                                                   const float* __restrict__ samples,
                                                   const uint32_t* __restrict__ hist,
                                                   const float* __restrict__ cols, int64_t n,
                                                   int d, float* __restrict__ splitv)
{
    __shared__ uint32_t wsum[kWavesPerBlock];
    __shared__ long long gbest[kBlock];
    __shared__ float fl[kBlock], fh[kBlock];
    const int node = blockIdx.x, t = threadIdx.x;
    const int64_t start = lv_start[node], c = lv_count[node];
    const int s = (int)(c < kSampleMax ? c : kSampleMax);
    const int dim = dimv[node];
    if (dim >= 0) {
        // thread t owns bins 4t .. 4t+3; C_j = sum of bins 0..j
        uint32_t hb[4], sum = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int j = 4 * t + r;
            hb[r] = j < s ? hist[(int64_t)node * kBins + j] : 0u;
            sum += hb[r];
        }
        uint32_t tot;
        uint32_t C = block_excl_scan(sum, &tot, wsum);
        // key = gap * 2048 + j: the minimum gives the smallest gap, then smallest j
        long long key = LLONG_MAX;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int j = 4 * t + r;
            C += hb[r];
            if (j < s && C > 0 && (int64_t)C < c) {
                long long gap = 2 * (long long)C - c;
                if (gap < 0) gap = -gap;
                long long kk = gap * 2048 + j;
                if (kk < key) key = kk;
            }
        }
        gbest[t] = key;
        __syncthreads();
        for (int w = kBlock / 2; w >= 1; w >>= 1) {
            if (t < w && gbest[t + w] < gbest[t]) gbest[t] = gbest[t + w];
            __syncthreads();
        }
        if (t == 0) {
            // V > 0 guarantees a valid j; the guard only keeps the index in range
            int j = gbest[0] == LLONG_MAX ? 0 : (int)(gbest[0] % 2048);
            splitv[node] = samples[(int64_t)node * kSampleMax + j];
        }
        return;
    }
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
    if (t == 0) {
        dimv[node] = bd;  // -1 keeps a leaf
        splitv[node] = bhi;
    }
}

// ---------------------------------------------------------------------------
// B6: stable partition -- count, per-node scan, scatter
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_count(const int32_t* __restrict__ blk_node,
                                                  const int32_t* __restrict__ blk_begin,
                                                  const int32_t* __restrict__ lv_start,
                                                  const int32_t* __restrict__ lv_count,
                                                  const int32_t* __restrict__ dimv,
                                                  const float* __restrict__ splitv,
                                                  const float* __restrict__ cols, int64_t n,
                                                  uint32_t* __restrict__ wave_left)
{
    const int b = blockIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int node = blk_node[b];
    const int64_t start = lv_start[node], c = lv_count[node];
    const int64_t beg = blk_begin[b];
    const int64_t end = beg + kChunk < c ? beg + kChunk : c;
    const int64_t wb = beg + (int64_t)w * kWaveChunk;
    const int64_t we = wb + kWaveChunk < end ? wb + kWaveChunk : end;
    const int dim = dimv[node];
    uint32_t cnt = 0;
    if (dim < 0) {
        cnt = we > wb ? (uint32_t)(we - wb) : 0u;
    } else {
        const float split = splitv[node];
        const float* col = cols + (int64_t)dim * n + start;
        for (int64_t e0 = wb; e0 < we; e0 += kWave) {
            int64_t e = e0 + lane;
            bool f = e < we && col[e] < split;
            cnt += (uint32_t)__popcll(__ballot(f));
        }
    }
    if (lane == 0) wave_left[(int64_t)b * kWavesPerBlock + w] = cnt;
}

__global__ __launch_bounds__(kBlock) void k_blkscan(const int32_t* __restrict__ node_blk0,
                                                    const int32_t* __restrict__ node_nblk,
                                                    const uint32_t* __restrict__ wave_left,
                                                    uint32_t* __restrict__ blk_off,
                                                    int32_t* __restrict__ n_left)
{
    __shared__ uint32_t wsum[kWavesPerBlock];
    const int node = blockIdx.x, t = threadIdx.x;
    const int b0 = node_blk0[node], nb = node_nblk[node];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kBlock) {
        const int i = base + t;
        uint32_t v = 0;
        if (i < nb)
            for (int w = 0; w < kWavesPerBlock; ++w)
                v += wave_left[(int64_t)(b0 + i) * kWavesPerBlock + w];
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot, wsum);
        if (i < nb) blk_off[b0 + i] = carry + ex;
        carry += tot;
    }
    if (t == 0) n_left[node] = (int32_t)carry;
}

__global__ __launch_bounds__(kBlock) void k_scatter(
    const int32_t* __restrict__ blk_node, const int32_t* __restrict__ blk_begin,
    const int32_t* __restrict__ lv_start, const int32_t* __restrict__ lv_count,
    const int32_t* __restrict__ dimv, const float* __restrict__ splitv,
    const uint32_t* __restrict__ blk_off, const uint32_t* __restrict__ wave_left,
    const int32_t* __restrict__ n_left, const float* __restrict__ src_cols,
    const int32_t* __restrict__ src_idx, float* __restrict__ dst_cols,
    int32_t* __restrict__ dst_idx, int64_t n, int d)
{
    const int b = blockIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int node = blk_node[b];
    const int64_t start = lv_start[node], c = lv_count[node];
    const int64_t beg = blk_begin[b];
    const int64_t end = beg + kChunk < c ? beg + kChunk : c;
    const int64_t wb = beg + (int64_t)w * kWaveChunk;
    const int64_t we = wb + kWaveChunk < end ? wb + kWaveChunk : end;
    if (wb >= we) return;
    int64_t lefts_before = blk_off[b];
    for (int i = 0; i < w; ++i) lefts_before += wave_left[(int64_t)b * kWavesPerBlock + i];
    const int dim = dimv[node];
    const float split = splitv[node];
    const int64_t nl = n_left[node];
    int64_t base_l = start + lefts_before;
    int64_t base_r = start + nl + (wb - lefts_before);
    const float* key = dim >= 0 ? src_cols + (int64_t)dim * n + start : nullptr;
    for (int64_t e0 = wb; e0 < we; e0 += kWave) {
        const int64_t e = e0 + lane;
        const bool valid = e < we;
        const bool f = valid && (dim < 0 || key[e] < split);
        const uint64_t bl = __ballot(f), bv = __ballot(valid);
        if (valid) {
            const int64_t dst = f ? base_l + lanes_below(bl) : base_r + lanes_below(bv & ~bl);
            const int64_t src = start + e;
            for (int t = 0; t < d; ++t)
                dst_cols[(int64_t)t * n + dst] = src_cols[(int64_t)t * n + src];
            dst_idx[dst] = src_idx[src];
        }
        base_l += __popcll(bl);
        base_r += __popcll(bv & ~bl);
    }
}

// ---------------------------------------------------------------------------
// B8-B9: subtree finish, one wavefront per node of at most W points
// ---------------------------------------------------------------------------
struct SubEntry {
    int32_t start, count, node_id, parent;
    int32_t buf, leaf_only, depth0, pad;
};

__device__ inline void wave_bitonic(float* buf, int P, int lane)
{
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < P; i += kWave) {
                int ixj = i ^ j;
                if (ixj > i) {
                    float x = buf[i], y = buf[ixj];
                    bool asc = (i & k) == 0;
                    if ((x > y) == asc) {
                        buf[i] = y;
                        buf[ixj] = x;
                    }
                }
            }
            wave_sync();
        }
}

__global__ __launch_bounds__(kBlock) void k_finish(
    const SubEntry* __restrict__ subs, int32_t n_sub, const float* __restrict__ colsA,
    const int32_t* __restrict__ idxA, const float* __restrict__ colsB,
    const int32_t* __restrict__ idxB, int64_t n, int d, int leaf, int W, int max_depth,
    size_t per_wave, float* __restrict__ pts, NodeRec* __restrict__ tnodes,
    float* __restrict__ tbox, int32_t* __restrict__ sub_nodes, int32_t* __restrict__ err,
    int32_t* __restrict__ depth_seen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sub = blockIdx.x * kWavesPerBlock + w;
    if (sub >= n_sub) return;  // only wavefront-level synchronization below
    const SubEntry e = subs[sub];
    const float* cols = e.buf ? colsB : colsA;
    const int32_t* gidx = e.buf ? idxB : idxA;
    const int64_t gs = e.start;
    const int c = e.count;
    const int D2 = 2 * d;
    NodeRec* trec = tnodes + 2 * gs;
    float* tb = tbox + 2 * gs * D2;

    if (e.leaf_only || c <= leaf) {  // a bucket: box and packed rows straight from HBM
        for (int dd = 0; dd < d; ++dd) {
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
                tb[d + dd] = hi;
            }
        }
        for (int j = lane; j < c; j += kWave) {
            const int64_t row = (gs + j) * (d + 1);
            for (int dd = 0; dd < d; ++dd) pts[row + dd] = cols[(int64_t)dd * n + gs + j];
            pts[row + d] = __int_as_float(gidx[gs + j]);
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
    float* X = reinterpret_cast<float*>(region);                   // [d][W]
    uint16_t* perm = reinterpret_cast<uint16_t*>(X + (size_t)d * W);  // [W]
    float* sortbuf = reinterpret_cast<float*>(perm + W);            // [W] (also partition scratch)
    uint16_t* tmp = reinterpret_cast<uint16_t*>(sortbuf);
    int4* stack = reinterpret_cast<int4*>(sortbuf + W);             // [kStack]

    for (int dd = 0; dd < d; ++dd)
        for (int j = lane; j < c; j += kWave) X[dd * W + j] = cols[(int64_t)dd * n + gs + j];
    for (int j = lane; j < c; j += kWave) perm[j] = (uint16_t)j;
    if (lane == 0) {
        stack[0] = make_int4(0, 0, c, 0);
        trec[0].parent = -1;
    }
    wave_sync();
    int sp = 1, nloc = 1, maxdep = 0;
    bool bad = false;
    while (sp > 0) {
        const int4 top = stack[--sp];
        const int id = top.x, ls = top.y, lc = top.z, dep = top.w;
        if (dep > maxdep) maxdep = dep;
        // tight box of the node
        for (int dd = 0; dd < d; ++dd) {
            float lo = INFINITY, hi = -INFINITY;
            for (int j = lane; j < lc; j += kWave) {
                float x = X[dd * W + perm[ls + j]];
                lo = fminf(lo, x);
                hi = fmaxf(hi, x);
            }
            lo = wave_min(lo);
            hi = wave_max(hi);
            if (lane == 0) {
                tb[(int64_t)id * D2 + dd] = lo;
                tb[(int64_t)id * D2 + d + dd] = hi;
            }
        }
        bool make_leaf = lc <= leaf;
        int best = 0;
        float split = 0.0f;
        int nl = 0;
        if (!make_leaf) {
            // split dimension: FP64 variance of all node points (the sample)
            double bestV = -1.0;
            for (int dd = 0; dd < d; ++dd) {
                double a[16], q[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    int j = lane + kWave * r;
                    a[r] = j < lc ? (double)X[dd * W + perm[ls + j]] : 0.0;
                }
                double av[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) av[r] = a[r];
                const double S = wave_psum(av);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    int j = lane + kWave * r;
                    double wv = (double)lc * a[r] - S;
                    q[r] = j < lc ? wv * wv : 0.0;
                }
                const double V = wave_psum(q);
                if (V > bestV) {
                    bestV = V;
                    best = dd;
                }
            }
            if (!(bestV > 0.0)) make_leaf = true;  // all points coincide
        }
        if (make_leaf) {
            if (lane == 0) {
                trec[id].a = (int32_t)(gs + ls);
                trec[id].split = 0.0f;
                trec[id].dim = -lc;
            }
            wave_sync();
            continue;
        }
        // exact split: value of rank lc/2 or the next larger value, whichever
        // count below is closer to half (ties to the smaller value)
        int P = 1;
        while (P < lc) P <<= 1;
        for (int j = lane; j < P; j += kWave)
            sortbuf[j] = j < lc ? X[best * W + perm[ls + j]] : INFINITY;
        wave_sync();
        wave_bitonic(sortbuf, P, lane);
        const float vstar = sortbuf[lc / 2];
        int r_lo = 0, r_hi = 0;
        for (int j0 = 0; j0 < lc; j0 += kWave) {
            int j = j0 + lane;
            float x = j < lc ? sortbuf[j] : INFINITY;
            r_lo += __popcll(__ballot(j < lc && x < vstar));
            r_hi += __popcll(__ballot(j < lc && x <= vstar));
        }
        const float vnext = r_hi < lc ? sortbuf[r_hi] : vstar;
        wave_sync();  // sortbuf is reused as partition scratch below
        const bool ok_star = r_lo > 0, ok_next = r_hi < lc;
        if (ok_star && (!ok_next || (lc - 2 * r_lo) <= (2 * r_hi - lc))) {
            split = vstar;
            nl = r_lo;
        } else {
            split = vnext;
            nl = r_hi;
        }
        // stable partition of perm[ls .. ls+lc)
        int bl_run = 0, br_run = 0;
        for (int j0 = 0; j0 < lc; j0 += kWave) {
            const int j = j0 + lane;
            const bool valid = j < lc;
            const uint16_t p = valid ? perm[ls + j] : 0;
            const bool f = valid && X[best * W + p] < split;
            const uint64_t bl = __ballot(f), bv = __ballot(valid);
            if (valid) {
                int dst = f ? bl_run + (int)lanes_below(bl) : nl + br_run + (int)lanes_below(bv & ~bl);
                tmp[dst] = p;
            }
            bl_run += __popcll(bl);
            br_run += __popcll(bv & ~bl);
        }
        wave_sync();
        for (int j = lane; j < lc; j += kWave) perm[ls + j] = tmp[j];
        const int L = nloc, R = nloc + 1;
        nloc += 2;
        if (e.depth0 + dep + 1 > max_depth || sp + 2 > kStack) bad = true;
        if (lane == 0) {
            trec[id].a = L;
            trec[id].split = split;
            trec[id].dim = best;
            trec[L].parent = id;
            trec[R].parent = id;
            if (!bad) {
                const int4 lft = make_int4(L, ls, nl, dep + 1);
                const int4 rgt = make_int4(R, ls + nl, lc - nl, dep + 1);
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
        if (bad) break;
        sp += 2;
    }
    if (bad) {
        if (lane == 0) atomicExch(err, KNN_EDEPTH);
        return;
    }
    for (int j = lane; j < c; j += kWave) {
        const int p = perm[j];
        const int64_t row = (gs + j) * (d + 1);
        for (int dd = 0; dd < d; ++dd) pts[row + dd] = X[dd * W + p];
        pts[row + d] = __int_as_float(gidx[gs + p]);
    }
    if (lane == 0) {
        sub_nodes[sub] = nloc;
        atomicMax(depth_seen, e.depth0 + maxdep);
    }
}

// Final ids: subtree root keeps its level-pass id, local node j >= 1 becomes
// sub_base + j - 1.
__global__ __launch_bounds__(kBlock) void k_compact(const SubEntry* __restrict__ subs,
                                                    int32_t n_sub,
                                                    const int32_t* __restrict__ sub_nodes,
                                                    const int32_t* __restrict__ sub_base,
                                                    const NodeRec* __restrict__ tnodes,
                                                    const float* __restrict__ tbox, int d,
                                                    NodeRec* __restrict__ nodes,
                                                    float* __restrict__ bbox)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sub = blockIdx.x * kWavesPerBlock + w;
    if (sub >= n_sub) return;
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

__global__ void k_bbox_up(const int32_t* __restrict__ ids, int32_t cnt,
                          const NodeRec* __restrict__ nodes, float* __restrict__ bbox, int d)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const int v = ids[i];
    const int L = nodes[v].a;
    const int D2 = 2 * d;
    for (int t = 0; t < d; ++t) {
        bbox[(int64_t)v * D2 + t] = fminf(bbox[(int64_t)L * D2 + t], bbox[(int64_t)(L + 1) * D2 + t]);
        bbox[(int64_t)v * D2 + d + t] =
            fmaxf(bbox[(int64_t)L * D2 + d + t], bbox[(int64_t)(L + 1) * D2 + d + t]);
    }
}

struct LevelNode {
    int32_t start, count, id, parent, depth;
};

}  // namespace

size_t finish_lds_bytes_per_wave(int32_t d, int32_t w)
{
    // X [d][W] floats, perm [W] u16, sort/partition scratch [W] floats, stack
    size_t b = (size_t)4 * d * w + (size_t)2 * w + (size_t)4 * w + sizeof(int4) * kStack;
    return (b + 15) & ~(size_t)15;
}

int32_t default_subtree_points(int32_t d)
{
    // two blocks of four wavefronts per CU: at most 80 KiB of LDS per block
    int32_t w = kSampleMax;
    while (w > 64 && finish_lds_bytes_per_wave(d, w) * kWavesPerBlock > 80 * 1024) w >>= 1;
    return w;
}

int build_tree(const float* points, int64_t n, int32_t d, int32_t leaf, int32_t max_depth,
               int32_t W, hipStream_t st, knn_tree** out)
{
    prof_mark(st, 0);
    const int64_t nd = n * d;
    DevBuf colsA, colsB, idxA, idxB, pts;
    KNN_HIP(colsA.alloc(sizeof(float) * nd));
    KNN_HIP(colsB.alloc(sizeof(float) * nd));
    KNN_HIP(idxA.alloc(sizeof(int32_t) * n));
    KNN_HIP(idxB.alloc(sizeof(int32_t) * n));
    KNN_HIP(pts.alloc(sizeof(float) * n * (d + 1)));
    {
        int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 65536);
        k_ingest<<<(unsigned)blocks, kBlock, 0, st>>>(points, n, d, colsA.as<float>(),
                                                      idxA.as<int32_t>());
        KNN_HIP(hipGetLastError());
    }
    prof_mark(st, 1);

    // ---- level passes -------------------------------------------------------
    const int64_t nn_max = n / W + 1;
    const int64_t nb_max = n / kChunk + nn_max + 1;
    DevBuf lvbuf, dimv, splitv, nleft, samples, hist, wave_left, blk_off;
    KNN_HIP(lvbuf.alloc(sizeof(int32_t) * (4 * nn_max + 2 * nb_max)));
    KNN_HIP(dimv.alloc(sizeof(int32_t) * nn_max));
    KNN_HIP(splitv.alloc(sizeof(float) * nn_max));
    KNN_HIP(nleft.alloc(sizeof(int32_t) * nn_max));
    KNN_HIP(samples.alloc(sizeof(float) * kSampleMax * nn_max));
    KNN_HIP(hist.alloc(sizeof(uint32_t) * kBins * nn_max));
    KNN_HIP(wave_left.alloc(sizeof(uint32_t) * kWavesPerBlock * nb_max));
    KNN_HIP(blk_off.alloc(sizeof(uint32_t) * nb_max));

    std::vector<LevelNode> level, next;
    std::vector<SubEntry> subs;
    std::vector<NodeRec> big;          // records of level-pass nodes (by id)
    std::vector<std::vector<int32_t>> inner_by_depth;
    big.push_back(NodeRec{0, -1, 0.0f, 0});
    int32_t next_id = 1;
    // a node goes through the level passes only if it is both above the bucket
    // size and too large for one wavefront's LDS
    auto needs_level = [&](int64_t c) { return c > W && c > leaf; };
    if (!needs_level(n)) {
        subs.push_back(SubEntry{0, (int32_t)n, 0, -1, 0, 0, 0, 0});
    } else {
        level.push_back(LevelNode{0, (int32_t)n, 0, -1, 0});
    }
    int buf = 0;  // buffer holding the current level's points
    std::vector<int32_t> hbuf;
    std::vector<int32_t> h_dim;
    std::vector<float> h_split;
    std::vector<int32_t> h_nl;
    while (!level.empty()) {
        const int32_t nn = (int32_t)level.size();
        if (level[0].depth + 1 > max_depth)
            return fail(KNN_EDEPTH, "tree deeper than max_depth");
        // block table: each node's points in chunks of kChunk
        std::vector<int32_t> blk_node, blk_begin, node_blk0(nn), node_nblk(nn);
        for (int32_t i = 0; i < nn; ++i) {
            const int32_t nb = (int32_t)((level[i].count + kChunk - 1) / kChunk);
            node_blk0[i] = (int32_t)blk_node.size();
            node_nblk[i] = nb;
            for (int32_t j = 0; j < nb; ++j) {
                blk_node.push_back(i);
                blk_begin.push_back(j * kChunk);
            }
        }
        const int32_t nb = (int32_t)blk_node.size();
        hbuf.assign(4 * (size_t)nn + 2 * (size_t)nb, 0);
        for (int32_t i = 0; i < nn; ++i) {
            hbuf[i] = level[i].start;
            hbuf[nn + i] = level[i].count;
            hbuf[2 * nn + i] = node_blk0[i];
            hbuf[3 * nn + i] = node_nblk[i];
        }
        std::copy(blk_node.begin(), blk_node.end(), hbuf.begin() + 4 * nn);
        std::copy(blk_begin.begin(), blk_begin.end(), hbuf.begin() + 4 * nn + nb);
        KNN_HIP(hipMemcpyAsync(lvbuf.p, hbuf.data(), sizeof(int32_t) * hbuf.size(),
                               hipMemcpyHostToDevice, st));
        const int32_t* d_start = lvbuf.as<int32_t>();
        const int32_t* d_count = d_start + nn;
        const int32_t* d_blk0 = d_start + 2 * nn;
        const int32_t* d_nblk = d_start + 3 * nn;
        const int32_t* d_bnode = d_start + 4 * nn;
        const int32_t* d_bbeg = d_bnode + nb;
        const float* src = (buf ? colsB : colsA).as<float>();
        const int32_t* srci = (buf ? idxB : idxA).as<int32_t>();
        float* dst = (buf ? colsA : colsB).as<float>();
        int32_t* dsti = (buf ? idxA : idxB).as<int32_t>();

        k_sample<<<nn, kBlock, 0, st>>>(d_start, d_count, src, n, d, samples.as<float>(),
                                        dimv.as<int32_t>());
        KNN_HIP(hipMemsetAsync(hist.p, 0, sizeof(uint32_t) * kBins * (size_t)nn, st));
        k_hist<<<nb, kBlock, 0, st>>>(d_bnode, d_bbeg, d_start, d_count, dimv.as<int32_t>(),
                                      samples.as<float>(), src, n, hist.as<uint32_t>());
        k_choose<<<nn, kBlock, 0, st>>>(d_start, d_count, dimv.as<int32_t>(),
                                        samples.as<float>(), hist.as<uint32_t>(), src, n, d,
                                        splitv.as<float>());
        k_count<<<nb, kBlock, 0, st>>>(d_bnode, d_bbeg, d_start, d_count, dimv.as<int32_t>(),
                                       splitv.as<float>(), src, n, wave_left.as<uint32_t>());
        k_blkscan<<<nn, kBlock, 0, st>>>(d_blk0, d_nblk, wave_left.as<uint32_t>(),
                                         blk_off.as<uint32_t>(), nleft.as<int32_t>());
        k_scatter<<<nb, kBlock, 0, st>>>(d_bnode, d_bbeg, d_start, d_count, dimv.as<int32_t>(),
                                         splitv.as<float>(), blk_off.as<uint32_t>(),
                                         wave_left.as<uint32_t>(), nleft.as<int32_t>(), src,
                                         srci, dst, dsti, n, d);
        KNN_HIP(hipGetLastError());
        h_dim.resize(nn);
        h_split.resize(nn);
        h_nl.resize(nn);
        KNN_HIP(hipMemcpyAsync(h_dim.data(), dimv.p, sizeof(int32_t) * nn, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipMemcpyAsync(h_split.data(), splitv.p, sizeof(float) * nn, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipMemcpyAsync(h_nl.data(), nleft.p, sizeof(int32_t) * nn, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));

        next.clear();
        const int nbuf = buf ^ 1;
        for (int32_t i = 0; i < nn; ++i) {
            const LevelNode& v = level[i];
            if (h_dim[i] < 0) {  // identical points: an oversized bucket
                subs.push_back(SubEntry{v.start, v.count, v.id, v.parent, nbuf, 1, v.depth, 0});
                continue;
            }
            const int32_t nl = h_nl[i];
            if (nl <= 0 || nl >= v.count)
                return fail(KNN_EDEVICE, "level pass produced an empty child");
            const int32_t L = next_id, R = next_id + 1;
            next_id += 2;
            if ((int64_t)next_id > 2 * n) return fail(KNN_EDEVICE, "node id overflow");
            big.resize(next_id, NodeRec{0, -1, 0.0f, 0});
            big[v.id] = NodeRec{L, v.parent, h_split[i], h_dim[i]};
            if ((int)inner_by_depth.size() <= v.depth) inner_by_depth.resize(v.depth + 1);
            inner_by_depth[v.depth].push_back(v.id);
            const LevelNode kids[2] = {{v.start, nl, L, v.id, v.depth + 1},
                                       {v.start + nl, v.count - nl, R, v.id, v.depth + 1}};
            for (const LevelNode& ch : kids) {
                if (needs_level(ch.count)) next.push_back(ch);
                else subs.push_back(SubEntry{ch.start, ch.count, ch.id, ch.parent, nbuf, 0, ch.depth, 0});
            }
        }
        level.swap(next);
        buf = nbuf;
    }
    lvbuf.reset(); samples.reset(); hist.reset(); wave_left.reset(); blk_off.reset();
    prof_mark(st, 2);

    // ---- subtree finish -----------------------------------------------------
    const int32_t n_sub = (int32_t)subs.size();
    const int32_t n_big = next_id;
    DevBuf d_subs, tnodes, tbox, subn, flags;
    KNN_HIP(d_subs.alloc(sizeof(SubEntry) * n_sub));
    KNN_HIP(tnodes.alloc(sizeof(NodeRec) * 2 * n));
    KNN_HIP(tbox.alloc(sizeof(float) * 2 * n * 2 * d));
    KNN_HIP(subn.alloc(sizeof(int32_t) * n_sub));
    KNN_HIP(flags.alloc(sizeof(int32_t) * 2));
    KNN_HIP(hipMemcpyAsync(d_subs.p, subs.data(), sizeof(SubEntry) * n_sub, hipMemcpyHostToDevice, st));
    KNN_HIP(hipMemsetAsync(flags.p, 0, sizeof(int32_t) * 2, st));
    const size_t per_wave = finish_lds_bytes_per_wave(d, W);
    const size_t lds = per_wave * kWavesPerBlock;
    const int32_t fblocks = (n_sub + kWavesPerBlock - 1) / kWavesPerBlock;
    if (lds > 64 * 1024)
        KNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_finish),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    k_finish<<<fblocks, kBlock, lds, st>>>(
        d_subs.as<SubEntry>(), n_sub, colsA.as<float>(), idxA.as<int32_t>(), colsB.as<float>(),
        idxB.as<int32_t>(), n, d, leaf, W, max_depth, per_wave, pts.as<float>(),
        tnodes.as<NodeRec>(), tbox.as<float>(), subn.as<int32_t>(), flags.as<int32_t>(),
        flags.as<int32_t>() + 1);
    KNN_HIP(hipGetLastError());
    std::vector<int32_t> h_subn(n_sub);
    int32_t h_flags[2] = {0, 0};
    KNN_HIP(hipMemcpyAsync(h_subn.data(), subn.p, sizeof(int32_t) * n_sub, hipMemcpyDeviceToHost, st));
    KNN_HIP(hipMemcpyAsync(h_flags, flags.p, sizeof(h_flags), hipMemcpyDeviceToHost, st));
    KNN_HIP(hipStreamSynchronize(st));
    prof_mark(st, 3);
    if (h_flags[0] == KNN_EDEPTH) return fail(KNN_EDEPTH, "tree deeper than max_depth");
    if (h_flags[0]) return fail(KNN_EDEVICE, "subtree finish failed");

    // ---- ids, records, boxes --------------------------------------------------
    std::vector<int32_t> h_base(n_sub);
    int64_t total = n_big;
    int64_t leaves = 0;
    for (int32_t i = 0; i < n_sub; ++i) {
        h_base[i] = (int32_t)total;
        total += h_subn[i] - 1;
    }
    DevBuf nodes, bbox, d_base;
    KNN_HIP(nodes.alloc(sizeof(NodeRec) * total));
    KNN_HIP(bbox.alloc(sizeof(float) * total * 2 * d));
    KNN_HIP(d_base.alloc(sizeof(int32_t) * n_sub));
    KNN_HIP(hipMemcpyAsync(nodes.p, big.data(), sizeof(NodeRec) * n_big, hipMemcpyHostToDevice, st));
    KNN_HIP(hipMemcpyAsync(d_base.p, h_base.data(), sizeof(int32_t) * n_sub, hipMemcpyHostToDevice, st));
    k_compact<<<fblocks, kBlock, 0, st>>>(d_subs.as<SubEntry>(), n_sub, subn.as<int32_t>(),
                                          d_base.as<int32_t>(), tnodes.as<NodeRec>(),
                                          tbox.as<float>(), d, nodes.as<NodeRec>(),
                                          bbox.as<float>());
    KNN_HIP(hipGetLastError());
    DevBuf d_ids;
    size_t max_ids = 1;
    for (auto& v : inner_by_depth) max_ids = std::max(max_ids, v.size());
    KNN_HIP(d_ids.alloc(sizeof(int32_t) * max_ids));
    for (int dep = (int)inner_by_depth.size() - 1; dep >= 0; --dep) {
        const auto& ids = inner_by_depth[dep];
        if (ids.empty()) continue;
        KNN_HIP(hipMemcpyAsync(d_ids.p, ids.data(), sizeof(int32_t) * ids.size(),
                               hipMemcpyHostToDevice, st));
        k_bbox_up<<<(unsigned)((ids.size() + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            d_ids.as<int32_t>(), (int32_t)ids.size(), nodes.as<NodeRec>(), bbox.as<float>(), d);
        KNN_HIP(hipGetLastError());
    }
    KNN_HIP(hipStreamSynchronize(st));
    prof_mark(st, 4);

    knn_tree* t = new knn_tree();
    t->n = n;
    t->d = d;
    t->leaf = leaf;
    t->depth = h_flags[1];
    t->sub_pts = W;
    t->n_nodes = total;
    (void)leaves;
    (void)hipGetDevice(&t->device);
    t->bytes = (int64_t)(pts.bytes + nodes.bytes + bbox.bytes);
    t->pts = pts.as<float>();
    t->nodes = nodes.as<NodeRec>();
    t->bbox = bbox.as<float>();
    pts.release();
    nodes.release();
    bbox.release();
    *out = t;
    return KNN_OK;
}

}  // namespace knn
