// reduce.hip -- dispatch of the reduction kernels (reduce_kernels.hpp) by
// element type.
#include "reduce_kernels.hpp"

namespace salt {

int64_t reduce_tile_elems(int dtype) {
    switch (dtype) {
        case SALT_F64: return tile_elems<SALT_F64>();
        case SALT_F32: return tile_elems<SALT_F32>();
        case SALT_BF16: return tile_elems<SALT_BF16>();
        case SALT_F16: return tile_elems<SALT_F16>();
        default: return 0;
    }
}

hipError_t launch_reduce(const ReduceLaunch &L, int dtype) {
    switch (dtype) {
        case SALT_F64: return launch_reduce_f64(L);
        case SALT_F32: return launch_reduce_f32(L);
        case SALT_BF16: return launch_reduce_bf16(L);
        case SALT_F16: return launch_reduce_f16(L);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_expr(const ReduceExprLaunch &L, const Program &px, const Program *py, int dtype) {
    switch (dtype) {
        case SALT_F64: return launch_reduce_expr_f64(L, px, py);
        case SALT_F32: return launch_reduce_expr_f32(L, px, py);
        case SALT_BF16: return launch_reduce_expr_bf16(L, px, py);
        case SALT_F16: return launch_reduce_expr_f16(L, px, py);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_tree(const ReduceExprLaunch &L, int id, int dtype) {
    switch (dtype) {
        case SALT_F64: return launch_reduce_tree_f64(L, id);
        case SALT_F32: return launch_reduce_tree_f32(L, id);
        case SALT_BF16: return launch_reduce_tree_bf16(L, id);
        case SALT_F16: return launch_reduce_tree_f16(L, id);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace salt
