// batch.hpp -- the device descriptor of one batched item, shared by the host
// planner (api) and the batched kernels.
#pragma once

#include <cstdint>

#include "salt.h"

namespace salt {

// One item of a batched launch, in the canonical operand order of the
// batch's program. 256 bytes, so the table is an array of aligned records.
struct alignas(16) DevItem {
    int64_t n;
    int64_t tile_begin;  // first global tile of this item
    int32_t vec;         // every array of the item is 16-byte aligned
    int32_t tree;        // catalogue id of the item's tree (mixed-tree launches)
    const void *ops[SALT_MAX_OPERANDS];
    double sc64[SALT_MAX_SCALARS];  // scalars rounded to binary64 ...
    float sc32[SALT_MAX_SCALARS];   // ... and to binary32 (once, on the host)
    void *out;      // element-wise output, or null
    void *dot_out;  // dot of canonical operands 0 and 1, or null
    int64_t pad1[7];
};
static_assert(sizeof(DevItem) == 256, "descriptor layout");

// One entry of the execution list: tile `tile` of item `item`. Its partial
// goes to ws[items[item].tile_begin + tile], whatever its place in the list.
struct TileRef {
    int32_t item;
    int32_t tile;
};

// Order of the execution list: full tiles first, then the items' ragged last
// tiles by decreasing length (longest processing time first), so the grid's
// last workgroups are the light ones.
void order_tiles(TileRef *refs, int64_t count, const DevItem *items, int64_t tile_elems);

// Host-side launch of the batched kernels for one (tree, dtype).
struct BatchLaunch {
    const DevItem *items;
    const TileRef *tiles;  // execution list (or a consecutive range of it)
    int64_t total_tiles;   // entries of `tiles` this launch runs
    int32_t count;
    int32_t any_dot;
    double *ws;  // one binary64 partial per global tile (when any_dot)
    int32_t unroll;
    int32_t nontemporal;
    int64_t blocks;
    void *stream;
    int32_t combine;  // when any_dot: run the per-item combine after the kernel
                      // (0 for every range of a split list but the last)
};

using BatchFn = int (*)(const BatchLaunch &);  // returns a hipError_t
BatchFn catalogue_batch_launcher(int id, int dtype);
// Launcher for items of any catalogue trees in one element type: each item
// names its tree (DevItem::tree); element-wise evaluation only (no dot).
BatchFn catalogue_batch_multi_launcher(int dtype);
// Number of distinct operands the catalogue tree reads (-1: bad id).
int catalogue_loads(int id);
// The per-item combine of the dots' partials alone (after a batched kernel
// that wrote them), for element type dtype.
BatchFn batch_combine_launcher(int dtype);

}  // namespace salt
