// batch.hip -- dispatch of the batched kernels (batch_kernels.hpp) by
// element type and catalogue tree.
#include "batch.hpp"
#include "expr.hpp"

namespace salt {

BatchFn batch_launcher_f64(int id);
BatchFn batch_launcher_f32(int id);
BatchFn batch_launcher_bf16(int id);
BatchFn batch_launcher_f16(int id);

BatchFn catalogue_batch_launcher(int id, int dtype) {
    switch (dtype) {
        case SALT_F64: return batch_launcher_f64(id);
        case SALT_F32: return batch_launcher_f32(id);
        case SALT_BF16: return batch_launcher_bf16(id);
        case SALT_F16: return batch_launcher_f16(id);
        default: return nullptr;
    }
}

int catalogue_loads(int id) {
    switch (id) {
#define SALT_CAT_CASE(name, ...) \
    case cat::id_##name: return cat::name::n_loads;
        SALT_CATALOGUE(SALT_CAT_CASE)
#undef SALT_CAT_CASE
        default: return -1;
    }
}

}  // namespace salt
