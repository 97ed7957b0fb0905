/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for exact k-NN with
 * a kd-tree built by sampled medians (Patwary et al., "PANDA: Extreme Scale
 * Parallel K-Nearest Neighbor on Distributed Architectures", arXiv 1607.08220).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or constant with the GPU library, and the GPU library never calls it.
 *
 * What is computed (each function cites the passage it follows):
 *
 *   orc_bf32   The k-NN problem itself (Section I: the k points closest to a
 *              query) written out as brute force, with the distance fixed as
 *              the FP32 squared Euclidean distance summed left to right over
 *              the dimensions with separate multiply and add.
 *   orc_bf64   The same in FP64 arithmetic (for the 1e-6 relative cross-check).
 *   orc_build  The local kd-tree of Section III-A: split dimension of maximum
 *              sample variance (III-A1, "Choice of split dimension"), split
 *              point from a histogram of all node points over 1024 sorted
 *              sample points, taking the interval point closest to 50 %
 *              (III-A1, "Choice of split point"), index shuffle (III-A ii),
 *              leaves of at most `leaf` points (III-A1, "Choice of bucket
 *              size"), bucket packing (III-A iv).
 *   orc_query  Algorithm 1 (Section III-B/III-C), with the readings below.
 *
 * Readings where the paper is silent or its printed text is wrong:
 *   R1  Distances are squared FP32 (no sqrt; monotone-equivalent).
 *   R2  Ties are broken by the original input index: the result is the k
 *       smallest (D, index) keys in lexicographic order.
 *   R3  After a heap replace, r' becomes the new maximum of the heap (the
 *       printed step assigns the inserted point's distance, which is wrong
 *       whenever that point is not the new maximum).
 *   R4  The far child's bound is the exact distance from q to the far child's
 *       cell: the split dimension's offset REPLACES the offset inherited from
 *       an ancestor split on the same dimension (the printed step adds it,
 *       counting that dimension twice and pruning true neighbours).  Offsets
 *       are kept per dimension and the bound is re-summed left to right, so it
 *       never exceeds the FP32 distance of any point in the cell.
 *   R5  A node is expanded when its bound is <= r' (heap full) or < r (heap
 *       not full); a point enters when (D, i) < top(H), or D < r while the
 *       heap holds fewer than k entries.  Candidates with D >= r never enter.
 *   R6  Near child: left iff q[dim] < split; equal goes right, matching the
 *       partition (x[dim] < split goes left, stable).
 *   R7  Sample: s = min(1024, cnt) points at positions
 *       lo + floor((2j+1) cnt / (2s)) of the node's current order.
 *       Variance of dimension t is evaluated, without division, as
 *       V_t = psum_j (s*v_j - psum_j v_j)^2 in FP64, where psum pads to a
 *       power of two P with zeros and adds a[i] += a[i+w] for w = P/2 .. 1.
 *       Split dimension = first argmax of V_t.
 *   R8  Split point: sorted sample s_0 <= ... <= s_{s-1}; each node point falls
 *       in bin #{j : s_j <= x}; C_j = #{x < s_j} is the running sum of bins;
 *       j* = first argmin |2 C_j - cnt| over 0 < C_j < cnt; split = s_{j*}.
 *   R9  If the sample is constant in every dimension (all V_t = 0): if the
 *       node's points are all identical it is a leaf (possibly oversized);
 *       otherwise split the dimension of largest extent (hi - lo, FP64,
 *       first argmax) at its maximum value.
 *   R10 Fewer than k candidates: pad with (+inf, -1).  self_ids[q] (if given,
 *       -1 = none) excludes exactly that input index.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#ifndef ORC_MUTANT
#define ORC_MUTANT 0 /* >0 plants a deliberate mistake; used only by the pin tests */
#endif

#define ORC_SAMPLE_MAX 1024

/* ------------------------------------------------------------------------ */
/* Distances                                                                 */
/* ------------------------------------------------------------------------ */

/* FP32 squared distance, left to right, separate multiply and add (R1). */
static float dist32(const float* q, const float* x, int d)
{
    float t = q[0] - x[0];
    float acc = t * t;
    for (int j = 1; j < d; ++j) {
        float u = q[j] - x[j];
        float sq = u * u;
#if ORC_MUTANT == 7
        acc = (float)((double)acc + (double)u * (double)u); /* fused-style rounding */
#else
        acc = acc + sq;
#endif
    }
    return acc;
}

/* FP64 squared distance of the FP32 inputs: the difference of two FP32 values
 * is exact in FP64 (for values within 2^29 of each other in magnitude), so
 * each term carries one rounding and the sum d - 1 more. */
static double dist64(const float* q, const float* x, int d)
{
#if ORC_MUTANT == 9
    float acc = 0.0f; /* accumulates in FP32 */
    for (int j = 0; j < d; ++j) {
        float u = q[j] - x[j];
        acc = acc + u * u;
    }
    return (double)acc;
#else
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        double u = (double)q[j] - (double)x[j];
        acc = acc + u * u;
    }
    return acc;
#endif
}

/* ------------------------------------------------------------------------ */
/* Bounded result list: sorted ascending by (D, i), at most k entries.       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int k, h;
    double* d; /* distances (float values are stored exactly) */
    int32_t* i;
} klist;

static int key_less(double da, int32_t ia, double db, int32_t ib)
{
#if ORC_MUTANT == 4
    return da < db || (da == db && ia > ib); /* reversed tie-break */
#else
    return da < db || (da == db && ia < ib);
#endif
}

/* Insert (D, i) keeping the list sorted; drops the maximum when already full. */
static void klist_insert(klist* L, double D, int32_t i)
{
    int p = (L->h < L->k) ? L->h : L->k - 1; /* slot freed for the newcomer */
    if (L->h < L->k) L->h++;
    while (p > 0 && key_less(D, i, L->d[p - 1], L->i[p - 1])) {
        L->d[p] = L->d[p - 1];
        L->i[p] = L->i[p - 1];
        --p;
    }
    L->d[p] = D;
    L->i[p] = i;
}

/* ------------------------------------------------------------------------ */
/* Brute force (the definition)                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    const float* X; int64_t n; int d;
    const float* Q; int64_t m; int k;
    const int32_t* self; double r2; int fp64;
    int32_t* oi; void* od;
    int64_t q0, q1;
    const struct orc_tree* tree;
    int64_t* stats;
} job_t;

static void bf_range(job_t* J)
{
    klist L;
    L.k = J->k;
    L.d = (double*)malloc(sizeof(double) * (size_t)J->k);
    L.i = (int32_t*)malloc(sizeof(int32_t) * (size_t)J->k);
    for (int64_t qi = J->q0; qi < J->q1; ++qi) {
        const float* q = J->Q + qi * J->d;
        int32_t self = J->self ? J->self[qi] : -1;
        L.h = 0;
        for (int64_t i = 0; i < J->n; ++i) {
            if ((int32_t)i == self) continue;
            double D = J->fp64 ? dist64(q, J->X + i * J->d, J->d)
                               : (double)dist32(q, J->X + i * J->d, J->d);
            if (!(D < J->r2)) continue; /* candidate set: D < r (R5) */
            if (L.h < L.k || key_less(D, (int32_t)i, L.d[L.k - 1], L.i[L.k - 1]))
                klist_insert(&L, D, (int32_t)i);
        }
        for (int j = 0; j < J->k; ++j) {
            int32_t idx = j < L.h ? L.i[j] : -1;
            double D = j < L.h ? L.d[j] : INFINITY;
            J->oi[qi * J->k + j] = idx;
            if (J->fp64) ((double*)J->od)[qi * J->k + j] = D;
            else ((float*)J->od)[qi * J->k + j] = (float)D;
        }
    }
    free(L.d);
    free(L.i);
}

static void* bf_thread(void* p) { bf_range((job_t*)p); return NULL; }

static int resolve_threads(int nthreads, int64_t m)
{
    if (nthreads <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        nthreads = c > 0 ? (int)c : 1;
    }
    if ((int64_t)nthreads > m) nthreads = (int)(m > 0 ? m : 1);
    return nthreads;
}

static int run_jobs(job_t proto, int nthreads, void* (*fn)(void*))
{
    nthreads = resolve_threads(nthreads, proto.m);
    job_t* jobs = (job_t*)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -2; }
    for (int t = 0; t < nthreads; ++t) { /* static partition of the queries */
        jobs[t] = proto;
        jobs[t].q0 = proto.m * t / nthreads;
        jobs[t].q1 = proto.m * (t + 1) / nthreads;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, fn, &jobs[t]);
    fn(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return 0;
}

static int check_common(int64_t n, int d, int64_t m, int k)
{
    if (n < 1 || d < 1 || d > 64 || m < 0 || k < 1) return -1;
    return 0;
}

/* Exact FP32 k-NN by brute force (Section I; readings R1, R2, R5, R10). */
int orc_bf32(const float* X, int64_t n, int d, const float* Q, int64_t m, int k,
             const int32_t* self_ids, float r2, int32_t* out_idx, float* out_d2,
             int nthreads)
{
    if (check_common(n, d, m, k)) return -1;
    if (m == 0) return 0;
    job_t J = {0};
    J.X = X; J.n = n; J.d = d; J.Q = Q; J.m = m; J.k = k;
    J.self = self_ids; J.r2 = (double)r2; J.fp64 = 0; J.oi = out_idx; J.od = out_d2;
    return run_jobs(J, nthreads, bf_thread);
}

/* The same in FP64 on the FP32 inputs, sorted by (D64, i). */
int orc_bf64(const float* X, int64_t n, int d, const float* Q, int64_t m, int k,
             const int32_t* self_ids, double r2, int32_t* out_idx, double* out_d2,
             int nthreads)
{
    if (check_common(n, d, m, k)) return -1;
    if (m == 0) return 0;
    job_t J = {0};
    J.X = X; J.n = n; J.d = d; J.Q = Q; J.m = m; J.k = k;
    J.self = self_ids; J.r2 = r2; J.fp64 = 1; J.oi = out_idx; J.od = out_d2;
    return run_jobs(J, nthreads, bf_thread);
}

/* FP32 distance of one pair, exported so tests can pin it against exact
 * rational arithmetic and its forward-error bound. */
float orc_dist32(const float* q, const float* x, int d) { return dist32(q, x, d); }

/* ------------------------------------------------------------------------ */
/* kd-tree build (Section III-A)                                             */
/* ------------------------------------------------------------------------ */

typedef struct orc_tree {
    int64_t n; int d; int leaf; int depth;
    int64_t n_nodes, cap;
    int32_t* dim;    /* split dimension, -1 for a leaf */
    float* split;    /* split value (inner nodes) */
    int64_t* left;   /* child ids, -1 for a leaf */
    int64_t* right;
    int64_t* start;  /* range of the node in packed order */
    int64_t* count;
    int32_t* level;
    float* lo;       /* tight bounding box [n_nodes][d] */
    float* hi;
    int32_t* perm;   /* packed order: perm[j] = original index */
    float* packed;   /* packed coordinates [n][d] (bucket packing, III-A iv) */
} orc_tree;

/* Fixed-shape pairwise sum (R7). */
static double psum(const double* v, int s, double* work)
{
    int P = 1;
    while (P < s) P *= 2;
    for (int i = 0; i < P; ++i) work[i] = i < s ? v[i] : 0.0;
    for (int w = P / 2; w >= 1; w /= 2)
        for (int i = 0; i < w; ++i) work[i] = work[i] + work[i + w];
    return work[0];
}

static int cmp_float(const void* a, const void* b)
{
    float x = *(const float*)a, y = *(const float*)b;
    return (x > y) - (x < y);
}

/* Number of sorted samples <= x (the histogram bin of x). */
static int bin_of(const float* sorted, int s, float x)
{
    int lo = 0, hi = s; /* first index with sorted[idx] > x */
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (sorted[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

typedef struct {
    const float* X; int d; int leaf; int max_depth;
    orc_tree* T;     /* node store the recursion appends to */
    int32_t* order; int32_t* tmp;
    double* sv; double* sq; double* work; float* sorted; int64_t* hist;
    int err;
    int spawn;       /* levels below which a right subtree may still get its own thread */
} build_ctx;

/* Double the node arrays of a store (only the stores of subtrees built by
 * other threads grow; the tree's own store is sized for 2n nodes). */
static int grow_store(orc_tree* T)
{
    int64_t cap = T->cap ? 2 * T->cap : 64;
    void* p[7];
    p[0] = realloc(T->dim, sizeof(int32_t) * (size_t)cap); if (p[0]) T->dim = (int32_t*)p[0];
    p[1] = realloc(T->split, sizeof(float) * (size_t)cap); if (p[1]) T->split = (float*)p[1];
    p[2] = realloc(T->left, sizeof(int64_t) * (size_t)cap); if (p[2]) T->left = (int64_t*)p[2];
    p[3] = realloc(T->right, sizeof(int64_t) * (size_t)cap); if (p[3]) T->right = (int64_t*)p[3];
    p[4] = realloc(T->start, sizeof(int64_t) * (size_t)cap); if (p[4]) T->start = (int64_t*)p[4];
    p[5] = realloc(T->count, sizeof(int64_t) * (size_t)cap); if (p[5]) T->count = (int64_t*)p[5];
    p[6] = realloc(T->level, sizeof(int32_t) * (size_t)cap); if (p[6]) T->level = (int32_t*)p[6];
    for (int i = 0; i < 7; ++i)
        if (!p[i]) return -1;
    T->cap = cap;
    return 0;
}

static int64_t new_node(build_ctx* B, int64_t start, int64_t cnt, int level)
{
    orc_tree* T = B->T;
    if (T->n_nodes == T->cap && grow_store(T)) { B->err = -2; return -1; }
    int64_t v = T->n_nodes++;
    T->dim[v] = -1; T->split[v] = 0.0f; T->left[v] = -1; T->right[v] = -1;
    T->start[v] = start; T->count[v] = cnt; T->level[v] = level;
    if (level > T->depth) T->depth = level;
    return v;
}

/* Choose (dim, split) for the node [lo, lo+c) of B->order; returns 0 when the
 * node must stay a leaf (all points identical). */
static int choose_split(build_ctx* B, int64_t lo, int64_t c, int* out_dim, float* out_split)
{
    const int d = B->d;
    const float* X = B->X;
    int s = c < ORC_SAMPLE_MAX ? (int)c : ORC_SAMPLE_MAX;
    int best = 0;
    double bestV = -1.0;
    for (int t = 0; t < d; ++t) {
        for (int j = 0; j < s; ++j) {
#if ORC_MUTANT == 8
            int64_t pos = lo + (int64_t)j * c / s; /* shifted sample positions */
#else
            int64_t pos = lo + ((int64_t)(2 * j + 1) * c) / (2 * (int64_t)s);
#endif
            B->sv[j] = (double)X[(int64_t)B->order[pos] * d + t];
        }
        double S = psum(B->sv, s, B->work);
        for (int j = 0; j < s; ++j) {
            double w = (double)s * B->sv[j] - S;
            B->sq[j] = w * w;
        }
        double V = psum(B->sq, s, B->work);
        if (V > bestV) { bestV = V; best = t; }
    }
    if (bestV > 0.0) {
        /* R8: histogram of all node points over the sorted sample. */
        for (int j = 0; j < s; ++j) {
            int64_t pos = lo + ((int64_t)(2 * j + 1) * c) / (2 * (int64_t)s);
#if ORC_MUTANT == 8
            pos = lo + (int64_t)j * c / s;
#endif
            B->sorted[j] = X[(int64_t)B->order[pos] * d + best];
        }
        qsort(B->sorted, (size_t)s, sizeof(float), cmp_float);
        for (int b = 0; b <= s; ++b) B->hist[b] = 0;
        for (int64_t p = lo; p < lo + c; ++p)
            B->hist[bin_of(B->sorted, s, X[(int64_t)B->order[p] * d + best])]++;
        int64_t C = 0, bestGap = -1;
        int jstar = -1;
        for (int j = 0; j < s; ++j) {
            C += B->hist[j]; /* C_j = #{x < s_j} */
            if (C <= 0 || C >= c) continue;
            int64_t gap = 2 * C - c;
            if (gap < 0) gap = -gap;
            if (bestGap < 0 || gap < bestGap) { bestGap = gap; jstar = j; }
        }
        /* V > 0 implies two distinct sample values, hence a valid j. */
        *out_dim = best;
        *out_split = B->sorted[jstar];
        return 1;
    }
    /* R9: the sample is constant in every dimension. */
    int bd = -1;
    double bext = 0.0;
    float bhi = 0.0f;
    for (int t = 0; t < d; ++t) {
        float mn = INFINITY, mx = -INFINITY;
        for (int64_t p = lo; p < lo + c; ++p) {
            float x = X[(int64_t)B->order[p] * d + t];
            if (x < mn) mn = x;
            if (x > mx) mx = x;
        }
        double ext = (double)mx - (double)mn;
        if (ext > bext) { bext = ext; bd = t; bhi = mx; }
    }
    if (bd < 0) return 0;
    *out_dim = bd;
    *out_split = bhi;
    return 1;
}

static void build_node(build_ctx* B, int64_t v);
static void build_children(build_ctx* B, int64_t L, int64_t R);

static void build_node(build_ctx* B, int64_t v)
{
    orc_tree* T = B->T;
    int64_t lo = T->start[v], c = T->count[v];
    if (B->err) return;
    if (c <= B->leaf) return; /* bucket-size rule */
    int dim;
    float split;
    if (!choose_split(B, lo, c, &dim, &split)) return; /* identical points: leaf */
    if (T->level[v] + 1 > B->max_depth) { B->err = -4; return; }
    /* Stable index shuffle: x[dim] < split to the left, order kept. */
    int64_t nl = 0, w = lo;
    for (int64_t p = lo; p < lo + c; ++p) {
        float x = B->X[(int64_t)B->order[p] * B->d + dim];
#if ORC_MUTANT == 5
        int goes_left = x <= split;
#else
        int goes_left = x < split;
#endif
        if (goes_left) { B->tmp[w++] = B->order[p]; nl++; }
    }
    for (int64_t p = lo; p < lo + c; ++p) {
        float x = B->X[(int64_t)B->order[p] * B->d + dim];
#if ORC_MUTANT == 5
        int goes_left = x <= split;
#else
        int goes_left = x < split;
#endif
        if (!goes_left) B->tmp[w++] = B->order[p];
    }
    if (nl == 0 || nl == c) return; /* cannot happen for a valid choice */
    memcpy(B->order + lo, B->tmp + lo, sizeof(int32_t) * (size_t)c);
    T->dim[v] = dim;
    T->split[v] = split;
    int64_t L = new_node(B, lo, nl, T->level[v] + 1);
    int64_t R = new_node(B, lo + nl, c - nl, T->level[v] + 1);
    if (B->err) return;
    T->left[v] = L;
    T->right[v] = R;
    build_children(B, L, R);
}

/* ---- optional threads: the two children of a node cover disjoint ranges of
 * the index order, so the right subtree can be built by another thread into
 * a store of its own.  Appending that store after the left subtree gives every
 * node the id the one-thread recursion gives it (left subtree first, then the
 * right one), so the tree is the same with any thread count. */

typedef struct {
    build_ctx ctx;  /* its T: a store whose node 0 stands for the right child */
    int64_t R;      /* the right child's id in the parent's store */
} fork_job;

static int ctx_scratch(build_ctx* B)
{
    B->sv = (double*)malloc(sizeof(double) * ORC_SAMPLE_MAX);
    B->sq = (double*)malloc(sizeof(double) * ORC_SAMPLE_MAX);
    B->work = (double*)malloc(sizeof(double) * ORC_SAMPLE_MAX);
    B->sorted = (float*)malloc(sizeof(float) * ORC_SAMPLE_MAX);
    B->hist = (int64_t*)malloc(sizeof(int64_t) * (ORC_SAMPLE_MAX + 1));
    return (B->sv && B->sq && B->work && B->sorted && B->hist) ? 0 : -1;
}

static void ctx_free_scratch(build_ctx* B)
{
    free(B->sv); free(B->sq); free(B->work); free(B->sorted); free(B->hist);
}

static void store_free(orc_tree* S)
{
    free(S->dim); free(S->split); free(S->left); free(S->right);
    free(S->start); free(S->count); free(S->level);
}

static void* fork_main(void* p)
{
    fork_job* J = (fork_job*)p;
    build_node(&J->ctx, 0);
    return NULL;
}

/* Append store S (node 0 = node R of B's store) to B's store. */
static void append_store(build_ctx* B, const orc_tree* S, int64_t R)
{
    orc_tree* T = B->T;
    int64_t base = T->n_nodes - 1; /* local id j >= 1 becomes base + j */
    while (T->cap < T->n_nodes + S->n_nodes - 1)
        if (grow_store(T)) { B->err = -2; return; }
    for (int64_t j = 0; j < S->n_nodes; ++j) {
        int64_t g = j == 0 ? R : base + j;
        T->dim[g] = S->dim[j];
        T->split[g] = S->split[j];
        T->left[g] = S->left[j] < 0 ? -1 : base + S->left[j];
        T->right[g] = S->right[j] < 0 ? -1 : base + S->right[j];
        T->start[g] = S->start[j];
        T->count[g] = S->count[j];
        T->level[g] = S->level[j];
    }
    T->n_nodes += S->n_nodes - 1;
    if (S->depth > T->depth) T->depth = S->depth;
}

static void build_children(build_ctx* B, int64_t L, int64_t R)
{
    orc_tree* T = B->T;
    if (B->spawn > 0) {
        fork_job* J = (fork_job*)calloc(1, sizeof(fork_job));
        orc_tree* S = (orc_tree*)calloc(1, sizeof(orc_tree));
        pthread_t th;
        if (J && S && ctx_scratch(&J->ctx) == 0 && grow_store(S) == 0) {
            J->ctx.X = B->X; J->ctx.d = B->d; J->ctx.leaf = B->leaf;
            J->ctx.max_depth = B->max_depth; J->ctx.order = B->order; J->ctx.tmp = B->tmp;
            J->ctx.T = S;
            J->ctx.spawn = B->spawn - 1;
            J->R = R;
            S->depth = T->level[R];
            S->n_nodes = 1;
            S->dim[0] = -1; S->split[0] = 0.0f; S->left[0] = -1; S->right[0] = -1;
            S->start[0] = T->start[R]; S->count[0] = T->count[R]; S->level[0] = T->level[R];
            if (pthread_create(&th, NULL, fork_main, J) == 0) {
                B->spawn--;
                build_node(B, L);
                B->spawn++;
                pthread_join(th, NULL);
                if (J->ctx.err) B->err = J->ctx.err;
                if (!B->err) append_store(B, S, R);
                ctx_free_scratch(&J->ctx);
                store_free(S);
                free(S);
                free(J);
                return;
            }
        }
        if (J) ctx_free_scratch(&J->ctx);
        if (S) store_free(S);
        free(S);
        free(J);
    }
    build_node(B, L);
    build_node(B, R);
}

void orc_tree_free(orc_tree* T)
{
    if (!T) return;
    free(T->dim); free(T->split); free(T->left); free(T->right);
    free(T->start); free(T->count); free(T->level); free(T->lo); free(T->hi);
    free(T->perm); free(T->packed);
    free(T);
}

/* Build the local kd-tree (Section III-A; readings R6-R9).  status: 0 ok,
 * -1 bad argument, -2 out of memory, -4 depth above max_depth.  nthreads > 1
 * builds subtrees of the top levels on their own threads (same tree). */
orc_tree* orc_build_mt(const float* X, int64_t n, int d, int leaf, int max_depth, int nthreads,
                       int* status)
{
    *status = -1;
    if (!X || n < 1 || d < 1 || d > 64 || leaf < 1 || max_depth < 0) return NULL;
    orc_tree* T = (orc_tree*)calloc(1, sizeof(orc_tree));
    if (!T) { *status = -2; return NULL; }
    T->n = n; T->d = d; T->leaf = leaf; T->cap = 2 * n;
    T->dim = (int32_t*)malloc(sizeof(int32_t) * (size_t)T->cap);
    T->split = (float*)malloc(sizeof(float) * (size_t)T->cap);
    T->left = (int64_t*)malloc(sizeof(int64_t) * (size_t)T->cap);
    T->right = (int64_t*)malloc(sizeof(int64_t) * (size_t)T->cap);
    T->start = (int64_t*)malloc(sizeof(int64_t) * (size_t)T->cap);
    T->count = (int64_t*)malloc(sizeof(int64_t) * (size_t)T->cap);
    T->level = (int32_t*)malloc(sizeof(int32_t) * (size_t)T->cap);
    T->perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    T->packed = (float*)malloc(sizeof(float) * (size_t)n * (size_t)d);
    build_ctx B = {0};
    B.X = X; B.d = d; B.leaf = leaf; B.max_depth = max_depth; B.T = T;
    for (int t = 1; t < nthreads; t *= 2) B.spawn++; /* 2^spawn subtrees run at once */
    B.tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!T->dim || !T->split || !T->left || !T->right || !T->start || !T->count ||
        !T->level || !T->perm || !T->packed || !B.tmp || ctx_scratch(&B)) {
        *status = -2;
        goto fail;
    }
    B.order = T->perm;
    for (int64_t i = 0; i < n; ++i) T->perm[i] = (int32_t)i;
    new_node(&B, 0, n, 0);
    build_node(&B, 0);
    if (B.err) { *status = B.err; goto fail; }
    /* Bucket packing (III-A iv) and tight boxes over each node's range. */
    for (int64_t j = 0; j < n; ++j)
        memcpy(T->packed + j * d, X + (int64_t)T->perm[j] * d, sizeof(float) * (size_t)d);
    T->lo = (float*)malloc(sizeof(float) * (size_t)T->n_nodes * (size_t)d);
    T->hi = (float*)malloc(sizeof(float) * (size_t)T->n_nodes * (size_t)d);
    if (!T->lo || !T->hi) { *status = -2; goto fail; }
    for (int64_t v = 0; v < T->n_nodes; ++v)
        for (int t = 0; t < d; ++t) {
            float mn = INFINITY, mx = -INFINITY;
            for (int64_t j = T->start[v]; j < T->start[v] + T->count[v]; ++j) {
                float x = T->packed[j * d + t];
                if (x < mn) mn = x;
                if (x > mx) mx = x;
            }
            T->lo[v * d + t] = mn;
            T->hi[v * d + t] = mx;
        }
    free(B.tmp);
    ctx_free_scratch(&B);
    *status = 0;
    return T;
fail:
    free(B.tmp);
    ctx_free_scratch(&B);
    orc_tree_free(T);
    return NULL;
}

orc_tree* orc_build(const float* X, int64_t n, int d, int leaf, int max_depth, int* status)
{
    return orc_build_mt(X, n, d, leaf, max_depth, 1, status);
}

int64_t orc_tree_nodes(const orc_tree* T) { return T->n_nodes; }
int orc_tree_depth(const orc_tree* T) { return T->depth; }

/* Copy the tree into caller arrays (any pointer may be NULL). */
void orc_tree_export(const orc_tree* T, int32_t* dim, float* split, int64_t* left,
                     int64_t* right, int64_t* start, int64_t* count, int32_t* level,
                     float* lo, float* hi, int32_t* perm, float* packed)
{
    size_t N = (size_t)T->n_nodes, d = (size_t)T->d, n = (size_t)T->n;
    if (dim) memcpy(dim, T->dim, N * sizeof(int32_t));
    if (split) memcpy(split, T->split, N * sizeof(float));
    if (left) memcpy(left, T->left, N * sizeof(int64_t));
    if (right) memcpy(right, T->right, N * sizeof(int64_t));
    if (start) memcpy(start, T->start, N * sizeof(int64_t));
    if (count) memcpy(count, T->count, N * sizeof(int64_t));
    if (level) memcpy(level, T->level, N * sizeof(int32_t));
    if (lo) memcpy(lo, T->lo, N * d * sizeof(float));
    if (hi) memcpy(hi, T->hi, N * d * sizeof(float));
    if (perm) memcpy(perm, T->perm, n * sizeof(int32_t));
    if (packed) memcpy(packed, T->packed, n * d * sizeof(float));
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (Section III-B step 2, Section III-C)                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t node;
    float bound; /* lower bound on D for every point of the node */
    float* off;  /* per-dimension offset of q from the node's cell (R4) */
} frame;

/* Heap-full / radius admission of a bound (R5). */
static int admissible(const klist* L, float b, double r2)
{
    if (L->h < L->k) return (double)b < r2;
#if ORC_MUTANT == 3
    return (double)b < L->d[L->k - 1]; /* strict: misses equal-distance ties */
#else
    return (double)b <= L->d[L->k - 1];
#endif
}

static void query_range(job_t* J)
{
    const orc_tree* T = J->tree;
    const int d = T->d, k = J->k;
    klist L;
    L.k = k;
    L.d = (double*)malloc(sizeof(double) * (size_t)k);
    L.i = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
    int cap = T->depth + 2;
    frame* S = (frame*)malloc(sizeof(frame) * (size_t)cap);
    float* offs = (float*)malloc(sizeof(float) * (size_t)cap * (size_t)d);
    float* cur = (float*)malloc(sizeof(float) * (size_t)d);
    for (int s = 0; s < cap; ++s) S[s].off = offs + (size_t)s * (size_t)d;
    for (int64_t qi = J->q0; qi < J->q1; ++qi) {
        const float* q = J->Q + qi * d;
        int32_t self = J->self ? J->self[qi] : -1;
        int64_t nodes = 0, leaves = 0, points = 0;
        L.h = 0;
        /* r' <- r; push (root, 0) */
        int sp = 0;
        S[0].node = 0;
        S[0].bound = 0.0f;
        for (int t = 0; t < d; ++t) S[0].off[t] = 0.0f;
        sp = 1;
        while (sp > 0) {
            frame* f = &S[--sp];
            int64_t v = f->node;
            float b = f->bound;
            memcpy(cur, f->off, sizeof(float) * (size_t)d); /* the slot is reused below */
            nodes++;
            if (T->dim[v] < 0) { /* leaf: scan the bucket */
                leaves++;
                for (int64_t j = T->start[v]; j < T->start[v] + T->count[v]; ++j) {
                    int32_t i = T->perm[j];
                    points++;
                    if (i == self) continue;
                    double D = (double)dist32(q, T->packed + j * d, d);
                    if (L.h < k) {
                        if (D < J->r2) klist_insert(&L, D, i);
                    } else if (key_less(D, i, L.d[k - 1], L.i[k - 1])) {
                        klist_insert(&L, D, i); /* r' = new maximum of H (R3) */
#if ORC_MUTANT == 1
                        L.d[k - 1] = D; /* printed step: r' takes the inserted distance */
#endif
                    }
                }
                continue;
            }
            if (!admissible(&L, b, J->r2)) continue;
            int t = T->dim[v];
            float sv = T->split[v];
            int q_left = q[t] < sv; /* near child is the left one (R6) */
            int64_t nearc = q_left ? T->left[v] : T->right[v];
            int64_t farc = q_left ? T->right[v] : T->left[v];
            float o = q_left ? sv - q[t] : q[t] - sv;
            float nb;
#if ORC_MUTANT == 2
            nb = b + o * o; /* printed step: adds on top of the inherited bound */
#else
            /* far child's cell: dimension t's offset is replaced (R4) */
            nb = 0.0f;
            for (int j = 0; j < d; ++j) {
                float oj = (j == t) ? o : cur[j];
                float sq = oj * oj;
                nb = (j == 0) ? sq : nb + sq;
            }
#endif
            if (admissible(&L, nb, J->r2)) { /* push (C2, d') */
                frame* g = &S[sp++];
                g->node = farc;
                g->bound = nb;
                memcpy(g->off, cur, sizeof(float) * (size_t)d);
                g->off[t] = o;
            }
            frame* h = &S[sp++]; /* push (C1, d): visited first */
            h->node = nearc;
            h->bound = b;
            memcpy(h->off, cur, sizeof(float) * (size_t)d);
        }
        for (int j = 0; j < k; ++j) {
            J->oi[qi * k + j] = j < L.h ? L.i[j] : -1;
            ((float*)J->od)[qi * k + j] = j < L.h ? (float)L.d[j] : INFINITY;
        }
        if (J->stats) {
            J->stats[qi * 3 + 0] = nodes;
            J->stats[qi * 3 + 1] = leaves;
            J->stats[qi * 3 + 2] = points;
        }
    }
    free(cur);
    free(offs);
    free(S);
    free(L.d);
    free(L.i);
}

static void* query_thread(void* p) { query_range((job_t*)p); return NULL; }

/* k-NN of m queries by Algorithm 1 on the tree (readings R1-R6, R10).
 * stats (nullable): per query [nodes popped, leaves scanned, points scanned]. */
int orc_query(const orc_tree* T, const float* Q, int64_t m, int k, const int32_t* self_ids,
              float r2, int32_t* out_idx, float* out_d2, int nthreads, int64_t* stats)
{
    if (!T || check_common(T->n, T->d, m, k)) return -1;
    if (m == 0) return 0;
    job_t J = {0};
    J.tree = T; J.d = T->d; J.n = T->n; J.Q = Q; J.m = m; J.k = k;
    J.self = self_ids; J.r2 = (double)r2; J.oi = out_idx; J.od = out_d2; J.stats = stats;
    return run_jobs(J, nthreads, query_thread);
}
