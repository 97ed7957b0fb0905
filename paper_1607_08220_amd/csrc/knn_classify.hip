// k-NN classification and regression on a query's neighbour list: the
// baseline method the paper applies to its labelled data (a majority vote of
// the k neighbours, Section V-C) and the regression form it names beside
// classification (Section I).  One thread per query.
#include <hip/hip_runtime.h>

#include <cmath>

#include "knn_internal.h"

namespace {

constexpr int kBlockC = 256;

// Majority label among the neighbours idx[0..k) (ascending distance, -1 =
// none): the label with the most votes; between labels with equally many, the
// one whose first neighbour comes first (is nearer).  -1 with no neighbour.
__global__ __launch_bounds__(kBlockC) void k_vote(const int32_t* __restrict__ idx, int64_t m,
                                                  int k, const int32_t* __restrict__ labels,
                                                  int32_t* __restrict__ out_class,
                                                  int32_t* __restrict__ out_votes)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= m) return;
    const int32_t* row = idx + q * k;
    int cnt = 0;
    while (cnt < k && row[cnt] >= 0) ++cnt;
    int best = -1, best_votes = 0;
    for (int j = 0; j < cnt; ++j) {
        const int32_t c = labels[row[j]];
        int first = j, votes = 0;
        for (int i = 0; i < cnt; ++i) {
            if (labels[row[i]] == c) {
                ++votes;
                first = i < first ? i : first;
            }
        }
        if (first == j && votes > best_votes) {  // each label once, at its nearest neighbour
            best = c;
            best_votes = votes;
        }
    }
    out_class[q] = best;
    if (out_votes) out_votes[q] = best_votes;
}

// Mean of the neighbours' values: FP32 sum in neighbour order (left to
// right, separate adds) divided by the neighbour count; NaN with none.
__global__ __launch_bounds__(kBlockC) void k_regress(const int32_t* __restrict__ idx, int64_t m,
                                                     int k, const float* __restrict__ values,
                                                     float* __restrict__ out)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= m) return;
    const int32_t* row = idx + q * k;
    float acc = 0.0f;
    int cnt = 0;
    for (int j = 0; j < k && row[j] >= 0; ++j) {
        acc = cnt == 0 ? values[row[j]] : acc + values[row[j]];
        ++cnt;
    }
    out[q] = cnt ? acc / (float)cnt : NAN;
}

}  // namespace

extern "C" {

int knn_classify(const int32_t* idx, int64_t m, int32_t k, const int32_t* labels,
                 int32_t* out_class, int32_t* out_votes, void* stream)
{
    if (m < 0) return knn::fail(KNN_EINVAL, "m must be >= 0");
    if (k < 1 || k > KNN_MAX_K) return knn::fail(KNN_EINVAL, "k must be in [1, 64]");
    if (m == 0) return KNN_OK;
    if (!idx || !labels || !out_class) return knn::fail(KNN_EINVAL, "NULL pointer");
    const unsigned grid = (unsigned)((m + kBlockC - 1) / kBlockC);
    hipLaunchKernelGGL(k_vote, dim3(grid), dim3(kBlockC), 0, static_cast<hipStream_t>(stream), idx,
                       m, k, labels, out_class, out_votes);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

int knn_regress(const int32_t* idx, int64_t m, int32_t k, const float* values, float* out,
                void* stream)
{
    if (m < 0) return knn::fail(KNN_EINVAL, "m must be >= 0");
    if (k < 1 || k > KNN_MAX_K) return knn::fail(KNN_EINVAL, "k must be in [1, 64]");
    if (m == 0) return KNN_OK;
    if (!idx || !values || !out) return knn::fail(KNN_EINVAL, "NULL pointer");
    const unsigned grid = (unsigned)((m + kBlockC - 1) / kBlockC);
    hipLaunchKernelGGL(k_regress, dim3(grid), dim3(kBlockC), 0, static_cast<hipStream_t>(stream),
                       idx, m, k, values, out);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

}  // extern "C"
