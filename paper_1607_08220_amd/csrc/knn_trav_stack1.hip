// Instantiations of the lane-per-query traversal with Algorithm 1's explicit
// stack in LDS (k_traverse_stack in knn_traverse.h) for dimensions 1 to
// 8; split from the other dimensions only so that the library compiles in
// parallel.
#include "knn_traverse.h"

namespace knn {
namespace {

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

}  // namespace

StackFn stack_for_low(int d, int k, bool stats)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return stats ? pick_stack<DD, true>(k) : pick_stack<DD, false>(k);
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4) KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
}

}  // namespace knn
