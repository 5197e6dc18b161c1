// batch.hip -- dispatch of the batched kernels (batch_kernels.hpp) by
// element type and catalogue tree.
#include <algorithm>

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

BatchFn batch_multi_launcher_f64();
BatchFn batch_multi_launcher_f32();
BatchFn batch_multi_launcher_bf16();
BatchFn batch_multi_launcher_f16();

BatchFn catalogue_batch_multi_launcher(int dtype) {
    switch (dtype) {
        case SALT_F64: return batch_multi_launcher_f64();
        case SALT_F32: return batch_multi_launcher_f32();
        case SALT_BF16: return batch_multi_launcher_bf16();
        case SALT_F16: return batch_multi_launcher_f16();
        default: return nullptr;
    }
}

BatchFn batch_combine_launcher_f64();
BatchFn batch_combine_launcher_f32();
BatchFn batch_combine_launcher_bf16();
BatchFn batch_combine_launcher_f16();

BatchFn batch_combine_launcher(int dtype) {
    switch (dtype) {
        case SALT_F64: return batch_combine_launcher_f64();
        case SALT_F32: return batch_combine_launcher_f32();
        case SALT_BF16: return batch_combine_launcher_bf16();
        case SALT_F16: return batch_combine_launcher_f16();
        default: return nullptr;
    }
}

void order_tiles(TileRef *refs, int64_t count, const DevItem *items, int64_t tile_elems) {
    auto weight = [&](const TileRef &r) {
        const int64_t rest = items[r.item].n - (int64_t)r.tile * tile_elems;
        return rest < tile_elems ? rest : tile_elems;
    };
    std::stable_sort(refs, refs + count, [&](const TileRef &a, const TileRef &b) { return weight(a) > weight(b); });
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
