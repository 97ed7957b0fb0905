// Instantiations of the team-of-lanes-per-query traversal (k_traverse_team in
// knn_traverse.h) for every dimension and teams of 8, 16 and 32 lanes.
#include "knn_traverse.h"

namespace knn {
namespace {

template <int D>
TraverseFn pick_team(int t)
{
    if (t == 8) return k_traverse_team<D, 8>;
    if (t == 16) return k_traverse_team<D, 16>;
    if (t == 32) return k_traverse_team<D, 32>;
    return nullptr;
}

}  // namespace

TraverseFn team_for(int d, int t)
{
    switch (d) {
#define KNN_DIM_CASE(DD) \
    case DD:             \
        return pick_team<DD>(t);
        KNN_DIM_CASE(1) KNN_DIM_CASE(2) KNN_DIM_CASE(3) KNN_DIM_CASE(4)
        KNN_DIM_CASE(5) KNN_DIM_CASE(6) KNN_DIM_CASE(7) KNN_DIM_CASE(8)
        KNN_DIM_CASE(9) KNN_DIM_CASE(10) KNN_DIM_CASE(11) KNN_DIM_CASE(12)
        KNN_DIM_CASE(13) KNN_DIM_CASE(14) KNN_DIM_CASE(15) KNN_DIM_CASE(16)
#undef KNN_DIM_CASE
    default:
        return nullptr;
    }
}

}  // namespace knn
