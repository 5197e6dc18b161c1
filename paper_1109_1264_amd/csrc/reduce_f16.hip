// reduce_f16.hip -- the reduction kernels for one element type (compiled
// separately so the types build in parallel).
#include "reduce_kernels.hpp"

namespace salt {
hipError_t launch_reduce_f16(const ReduceLaunch &L) { return launch_reduce_dt<SALT_F16>(L); }
hipError_t launch_reduce_expr_f16(const ReduceExprLaunch &L, const Program &px, const Program *py) {
    return launch_reduce_expr_dt<SALT_F16>(L, px, py);
}
hipError_t launch_reduce_tree_f16(const ReduceExprLaunch &L, int id) { return launch_reduce_tree_dt<SALT_F16>(L, id); }
}  // namespace salt
