// batch_device.hpp -- many independent expression evaluations (and dot products)
// of uneven length in one persistent launch (device code).
//
// Every item is cut into the reduction's fixed tiles (reduce_common.hpp),
// and the tiles of all items form one flat list. A grid of workgroups walks
// that list (grid-stride), so a 2^20-element item and a 64-element item cost
// in proportion to their tiles, and one launch replaces thousands. In each
// tile a lane loads its chunks of every operand in bursts, evaluates the tree
// and stores the result (the paper's load / operate / store packages,
// Sec. 4.3), and, when the item asks for it, accumulates dot(operand 0,
// operand 1) from the same registers: the operands are read once for both.
// The dot's accumulation order inside a tile and the combine over the item's
// tiles are exactly those of salt_dot, so an item's dot has the same bits in
// a batch as alone. A second small kernel combines each item's partials, one
// wave per item.
//
// Device code only: the library instantiates it for its catalogue trees
// (batch_kernels.hpp), and the run-time compiler (jit.hip) for any other
// tree, from this same text.
#pragma once

#include "batch.hpp"
#include "device.hpp"
#include "expr.hpp"
#include "reduce_common.hpp"

namespace salt {

template <int DT, int NL, int U, int NS>
struct BChunkCtx {
    using C = typename Tr<DT>::C;
    const u32x4 (&raw)[NL][U];
    const C (&s)[NS];
    int u, p;
    template <int K>
    __device__ __forceinline__ C ld() const { return Tr<DT>::get(raw[K][u], p); }
    template <int J>
    __device__ __forceinline__ C sc() const { return s[J]; }
};

// Operand and output pointers of an item are read from its descriptor in
// memory, so the compiler cannot tell their address space and would emit flat
// memory instructions (which also count against the LDS/scalar wait counter
// and force full waits). These name the global address space.
using gu32x4 = __attribute__((address_space(1))) u32x4;
template <bool NT>
__device__ __forceinline__ u32x4 gld16(const void *p, int64_t ci) {
    const gu32x4 *g = (const gu32x4 *)p + ci;
    if constexpr (NT) return __builtin_nontemporal_load(g);
    else return *g;
}
template <bool NT>
__device__ __forceinline__ void gst16(void *p, int64_t ci, u32x4 v) {
    gu32x4 *g = (gu32x4 *)p + ci;
    if constexpr (NT) __builtin_nontemporal_store(v, g);
    else *g = v;
}

// Shape of one tile of one item.
enum TileForm {
    kWhole = 0,    // inside the item, arrays aligned: plain 16-byte accesses
    kRagged = 1,   // the item's last tile, arrays aligned: range-checked
                   // buffer accesses, plus one chunk that straddles the end
    kUnaligned = 2 // some array not 16-byte aligned: element by element
};

// One tile of one item. `c0` is this lane's first chunk of the tile, `m` the
// elements of the item from the tile's start (m >= tile size for kWhole).
// All forms visit the chunks and accumulate the dot in the same order and
// read zeros past the end, so the partial is the same whichever form runs.
template <class E, int DT, int UR, bool NT, bool DOT, int FORM, int NL, int NS>
__device__ __forceinline__ void batch_tile(const void *const (&op)[NL], const typename Tr<DT>::C (&s)[NS],
                                           void *out, int64_t n, int64_t t, int64_t m,
                                           Acc<DT> (&acc)[Tr<DT>::V]) {
    using C = typename Tr<DT>::C;
    using S = typename Tr<DT>::S;
    constexpr int V = Tr<DT>::V;
    constexpr int64_t T = tile_elems<DT>();
    const int64_t tile_chunk = t * ((int64_t)kBlock * kChunksPerLane);  // first chunk of the tile
    const int64_t c0 = tile_chunk + threadIdx.x;
    // kRagged: whole chunks in range, and the chunk (relative index) that
    // straddles the end, if any.
    const int32_t whole = (int32_t)(m / V);
    const int32_t straddle = (m % V) ? whole : -1;
    __amdgpu_buffer_rsrc_t rin[NL], rout;
    if constexpr (FORM == kRagged) {
#pragma unroll
        for (int q = 0; q < E::n_loads; ++q) rin[q] = rsrc((const S *)op[q] + t * T, whole * 16);
        if (out) rout = rsrc((S *)out + t * T, whole * 16);
    }
    // Chunk rows (kBlock chunks each) that hold elements of the item. Rows
    // past them would only read zeros and drop their stores, and adding the
    // product +0 leaves an accumulator's bits unchanged (it is never -0), so
    // a short last tile stops after its last burst with data.
    const int rows = FORM == kWhole ? kChunksPerLane
                                    : (int)(m < T ? (m + (int64_t)kBlock * V - 1) / ((int64_t)kBlock * V)
                                                  : (int64_t)kChunksPerLane);
    // Bursts are not unrolled: unrolled, the compiler hoisted the next
    // burst's loads and the kernel needed 240 registers instead of 147 (FP32,
    // 3 operands, 8 chunks) while running 1-3% slower.
#pragma unroll 1
    for (int it0 = 0; it0 < rows; it0 += UR) {
        u32x4 raw[NL][UR];
        // a row of a short tile past its last element is neither loaded nor
        // stored nor added (uniform test)
        const auto live = [&](int u) { return FORM == kWhole || it0 + u < rows; };
#pragma unroll
        for (int q = 0; q < E::n_loads; ++q)
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                const int64_t ci = c0 + (int64_t)(it0 + u) * kBlock;
                raw[q][u] = u32x4{0u, 0u, 0u, 0u};
                if (!live(u)) continue;
                if constexpr (FORM == kWhole) {
                    raw[q][u] = gld16<NT>(op[q], ci);
                } else if constexpr (FORM == kRagged) {
                    raw[q][u] = bld16<NT>(rin[q], (int32_t)(ci - tile_chunk) * 16);
                } else {
                    raw[q][u] = load_chunk_guarded<DT, NT>(op[q], ci, n, false);
                }
            }
        if constexpr (FORM == kRagged) {
            // The straddling chunk read zeros above; its lane reloads the
            // elements that exist. The burst and the wave tests are uniform.
#pragma unroll
            for (int u = 0; u < UR; ++u)
                if (straddle >= 0 && it0 + u == straddle / kBlock && (int)threadIdx.x == straddle % kBlock) {
#pragma unroll
                    for (int q = 0; q < E::n_loads; ++q)
                        raw[q][u] = load_chunk_guarded<DT, NT>(op[q], c0 + (int64_t)(it0 + u) * kBlock, n, false);
                }
        }
        if (out) {
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                if (!live(u)) continue;
                C r[V];
#pragma unroll
                for (int p = 0; p < V; ++p) r[p] = E::ev(BChunkCtx<DT, NL, UR, NS>{raw, s, u, p});
                const int64_t ci = c0 + (int64_t)(it0 + u) * kBlock;
                if constexpr (FORM == kWhole) {
                    gst16<NT>(out, ci, Tr<DT>::template pack<V>(r));
                } else if constexpr (FORM == kRagged) {
                    bst16<NT>(rout, (int32_t)(ci - tile_chunk) * 16, Tr<DT>::template pack<V>(r));
                    if (straddle >= 0 && it0 + u == straddle / kBlock && (int)threadIdx.x == straddle % kBlock) {
#pragma unroll
                        for (int p = 0; p < V; ++p)
                            if (ci * V + p < n) Tr<DT>::st1(out, ci * V + p, r[p]);
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < V; ++p)
                        if (ci * V + p < n) Tr<DT>::st1(out, ci * V + p, r[p]);
                }
            }
        }
        if constexpr (DOT) {
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                if (!live(u)) continue;
#pragma unroll
                for (int p = 0; p < V; ++p) acc[p].add(Tr<DT>::get(raw[0][u], p), Tr<DT>::get(raw[1][u], p));
            }
        }
    }
}

template <class E, int DT, int UR, bool NT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_batch(const DevItem *__restrict__ items,
                                                  const TileRef *__restrict__ tiles, int64_t total_tiles,
                                                  double *ws) {
    using C = typename Tr<DT>::C;
    constexpr int V = Tr<DT>::V;
    constexpr int64_t T = tile_elems<DT>();
    constexpr int NL = E::n_loads > 0 ? E::n_loads : 1;
    constexpr int NS = E::n_scal > 0 ? E::n_scal : 1;
    static_assert(!DOT || E::n_loads >= 2, "dot needs two operands");
    __shared__ double lds[kBlock / 64];
    for (int64_t gt = blockIdx.x; gt < total_tiles; gt += gridDim.x) {
        const int k = __builtin_amdgcn_readfirstlane(tiles[gt].item);
        const int64_t t = __builtin_amdgcn_readfirstlane(tiles[gt].tile);
        const DevItem &it = items[k];
        const int64_t n = it.n;
        const bool vec = it.vec != 0;
        const void *op[NL];
#pragma unroll
        for (int q = 0; q < NL; ++q) op[q] = it.ops[q];
        C s[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            if constexpr (DT == SALT_F64) s[j] = it.sc64[j];
            else s[j] = it.sc32[j];
        }
        Acc<DT> acc[V];
        const int64_t m = n - t * T;
        // Streaming (non-temporal) accesses pay off on whole tiles; the short
        // ragged tiles run faster with ordinary cached accesses (measured).
        if (!vec)
            batch_tile<E, DT, UR, NT, DOT, kUnaligned>(op, s, it.out, n, t, m, acc);
        else if (m >= T)
            batch_tile<E, DT, UR, NT, DOT, kWhole>(op, s, it.out, n, t, m, acc);
        else
            batch_tile<E, DT, UR, false, DOT, kRagged>(op, s, it.out, n, t, m, acc);
        if constexpr (DOT) {
            if (it.dot_out) {
                const double v = block_sum<kBlock / 64>(lane_value<DT>(acc), lds);
                if (threadIdx.x == 0) ws[it.tile_begin + t] = v;
            }
        }
    }
}

// Tile `t` of item `it` evaluated with the tree E (no dot): the item's
// operands and scalars, then the tile form.
template <class E, int DT, int UR, bool NT>
__device__ __forceinline__ void eval_item_tile(const DevItem &it, int64_t t) {
    using C = typename Tr<DT>::C;
    constexpr int V = Tr<DT>::V;
    constexpr int64_t T = tile_elems<DT>();
    constexpr int NL = E::n_loads > 0 ? E::n_loads : 1;
    constexpr int NS = E::n_scal > 0 ? E::n_scal : 1;
    const int64_t n = it.n;
    const void *op[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) op[q] = it.ops[q];
    C s[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if constexpr (DT == SALT_F64) s[j] = it.sc64[j];
        else s[j] = it.sc32[j];
    }
    Acc<DT> unused[V];
    const int64_t m = n - t * T;
    if (!it.vec)
        batch_tile<E, DT, UR, NT, false, kUnaligned>(op, s, it.out, n, t, m, unused);
    else if (m >= T)
        batch_tile<E, DT, UR, NT, false, kWhole>(op, s, it.out, n, t, m, unused);
    else
        batch_tile<E, DT, UR, false, false, kRagged>(op, s, it.out, n, t, m, unused);
}

// Items of different catalogue trees in one launch (one element type): the
// tile list mixes the items' tiles, and each tile branches on its item's
// tree. The branch is uniform over the workgroup (one tile per workgroup at
// a time), so it costs a scalar compare, and a serving batch needs one
// launch per element type instead of one per (tree, element type).
template <int DT, int UR, bool NT>
__global__ __launch_bounds__(kBlock) void k_batch_multi(const DevItem *__restrict__ items,
                                                        const TileRef *__restrict__ tiles, int64_t total_tiles) {
    for (int64_t gt = blockIdx.x; gt < total_tiles; gt += gridDim.x) {
        const int k = __builtin_amdgcn_readfirstlane(tiles[gt].item);
        const int64_t t = __builtin_amdgcn_readfirstlane(tiles[gt].tile);
        const DevItem &it = items[k];
        switch (__builtin_amdgcn_readfirstlane(it.tree)) {
#define SALT_CAT_CASE(name, ...) \
    case cat::id_##name: eval_item_tile<cat::name, DT, UR, NT>(it, t); break;
            SALT_CATALOGUE(SALT_CAT_CASE)
#undef SALT_CAT_CASE
            default: break;
        }
    }
}

// One wave per item: the combine of salt_dot's pass 2, wave-serialised.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_batch_combine(const DevItem *__restrict__ items, int count,
                                                          const double *ws) {
    constexpr int64_t T = tile_elems<DT>();
    constexpr int kWaves = kBlock / 64;
    for (int k = blockIdx.x * kWaves + (threadIdx.x >> 6); k < count; k += gridDim.x * kWaves) {
        const DevItem &it = items[k];
        if (!it.dot_out) continue;
        const double r = combine_partials_wave(ws + it.tile_begin, (it.n + T - 1) / T);
        if ((threadIdx.x & 63) == 0) store_result<DT, false>(it.dot_out, r);
    }
}

}  // namespace salt
