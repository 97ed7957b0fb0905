/*
 * Drives the CPU oracle (oracle/oracle.c, linked in) through every entry
 * point on small random and degenerate inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: brute force in FP32 and
 * FP64, the kd-tree build with one and several threads, Algorithm 1 queries
 * with self exclusion and a radius, and the tree export.  It also checks
 * that the kd-tree answers equal brute force and that both builds agree, so
 * that a silent memory error would show as a wrong answer as well.
 * Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_tree orc_tree;
int orc_bf32(const float*, int64_t, int, const float*, int64_t, int, const int32_t*, float,
             int32_t*, float*, int);
int orc_bf64(const float*, int64_t, int, const float*, int64_t, int, const int32_t*, double,
             int32_t*, double*, int);
orc_tree* orc_build(const float*, int64_t, int, int, int, int*);
orc_tree* orc_build_mt(const float*, int64_t, int, int, int, int, int*);
void orc_tree_free(orc_tree*);
int64_t orc_tree_nodes(const orc_tree*);
void orc_tree_export(const orc_tree*, int32_t*, float*, int64_t*, int64_t*, int64_t*, int64_t*,
                     int32_t*, float*, float*, int32_t*, float*);
int orc_query(const orc_tree*, const float*, int64_t, int, const int32_t*, float, int32_t*,
              float*, int, int64_t*);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

static int run_case(int64_t n, int d, int leaf, int k, int kind)
{
    const int64_t m = 37;
    float* X = malloc(sizeof(float) * n * d);
    float* Q = malloc(sizeof(float) * m * d);
    int32_t* self = malloc(sizeof(int32_t) * m);
    for (int64_t i = 0; i < n * d; ++i)
        X[i] = kind == 0 ? (float)urand() : kind == 1 ? (float)(int)(urand() * 4) : 0.5f;
    for (int64_t q = 0; q < m; ++q) {
        const int64_t src = (int64_t)(urand() * n);
        for (int j = 0; j < d; ++j) Q[q * d + j] = q % 2 ? X[src * d + j] : (float)urand();
        self[q] = q % 2 ? (int32_t)src : -1;
    }
    int32_t *bi = malloc(sizeof(int32_t) * m * k), *ki = malloc(sizeof(int32_t) * m * k);
    float *bd = malloc(sizeof(float) * m * k), *kd = malloc(sizeof(float) * m * k);
    int32_t* b64i = malloc(sizeof(int32_t) * m * k);
    double* b64d = malloc(sizeof(double) * m * k);
    int64_t* st = malloc(sizeof(int64_t) * m * 3);
    int bad = 0, status = 0;
    orc_tree* T1 = orc_build(X, n, d, leaf, 64, &status);
    orc_tree* T4 = orc_build_mt(X, n, d, leaf, 64, 4, &status);
    if (!T1 || !T4) {
        fprintf(stderr, "build failed: %d\n", status);
        return 1;
    }
    const int64_t N = orc_tree_nodes(T1);
    if (orc_tree_nodes(T4) != N) bad = 1;
    int32_t* dim1 = malloc(sizeof(int32_t) * N);
    int32_t* dim4 = malloc(sizeof(int32_t) * N);
    float *lo = malloc(sizeof(float) * N * d), *hi = malloc(sizeof(float) * N * d);
    int32_t* perm = malloc(sizeof(int32_t) * n);
    float* packed = malloc(sizeof(float) * n * d);
    int64_t* left = malloc(sizeof(int64_t) * N);
    orc_tree_export(T1, dim1, NULL, left, NULL, NULL, NULL, NULL, lo, hi, perm, packed);
    orc_tree_export(T4, dim4, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
    if (!bad && memcmp(dim1, dim4, sizeof(int32_t) * N)) bad = 2;
    const float radii[2] = {INFINITY, 0.05f};
    for (int r = 0; r < 2; ++r) {
        orc_bf32(X, n, d, Q, m, k, self, radii[r], bi, bd, 3);
        orc_bf64(X, n, d, Q, m, k, self, radii[r], b64i, b64d, 2);
        orc_query(T1, Q, m, k, self, radii[r], ki, kd, 3, st);
        if (memcmp(bi, ki, sizeof(int32_t) * m * k) || memcmp(bd, kd, sizeof(float) * m * k))
            bad = 3;
        orc_query(T4, Q, m, k, self, radii[r], ki, kd, 1, NULL);
        if (memcmp(bi, ki, sizeof(int32_t) * m * k)) bad = 4;
    }
    orc_tree_free(T1);
    orc_tree_free(T4);
    free(X); free(Q); free(self); free(bi); free(ki); free(bd); free(kd); free(b64i); free(b64d);
    free(st); free(dim1); free(dim4); free(lo); free(hi); free(perm); free(packed); free(left);
    if (bad) fprintf(stderr, "case n=%ld d=%d leaf=%d k=%d kind=%d: check %d failed\n", (long)n,
                     d, leaf, k, kind, bad);
    return bad;
}

int main(void)
{
    int fails = 0;
    const int dims[5] = {1, 2, 3, 7, 16};
    for (int a = 0; a < 5; ++a)
        for (int kind = 0; kind < 3; ++kind) {
            fails += run_case(2000 + 37 * a, dims[a], 1 + 7 * a, 1 + 6 * a, kind) != 0;
            fails += run_case(5, dims[a], 2, 9, kind) != 0;  /* k > n */
        }
    fails += run_case(3000, 3, 32, 64, 0) != 0;
    printf("%s: %d failing cases\n", fails ? "FAIL" : "ok", fails);
    return fails ? 1 : 0;
}
