// Instantiations of the lane-per-query stack-free traversal (k_traverse in
// knn_traverse.h) for dimensions 1 to 8; split from the other
// dimensions only so that the library compiles in parallel.
#include "knn_traverse.h"

namespace knn {
namespace {

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

}  // namespace

TraverseFn traverse_for_low(int d, int k, bool stats)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return stats ? pick_traverse<DD, true>(k) : pick_traverse<DD, false>(k);
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4) KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
}

}  // namespace knn
