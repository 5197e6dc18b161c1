// eval_tree.hpp -- the fused element-wise kernel for a compile-time
// expression tree (device code).
//
// One kernel pass evaluates a whole tree per element (loop fusion, Sec. 2):
// every operand is read once, the result written once, intermediates stay
// in registers. Each lane first issues all of its 16-byte loads for a tile
// (U chunks per operand), then evaluates the tree on the loaded registers,
// then issues all of its stores (the paper's instruction packages, Sec.
// 4.3). Elements after the last whole tile, and every element when an array
// is not 16-byte aligned, go through a per-element loop.
//
// The library instantiates it for its catalogue trees (eval.hip), and the
// run-time compiler (jit.hip) for any other tree, from this same text.
#pragma once

#include "device.hpp"
#include "expr.hpp"

namespace salt {

template <int DT>
struct EvalArgs {
    const void *ops[SALT_MAX_OPERANDS];
    typename Tr<DT>::C sc[SALT_MAX_SCALARS];
    void *out;
    int64_t n;
    int32_t vec;  // 1: 16-byte path for whole tiles; 0: per-element path only
};

// Operand values of one lane's tile: element p of chunk u of operand K.
template <int DT, int NL, int U, int NS>
struct ChunkCtx {
    using C = typename Tr<DT>::C;
    const u32x4 (&raw)[NL][U];
    const C (&s)[NS];
    int u, p;
    template <int K>
    __device__ __forceinline__ C ld() const { return Tr<DT>::get(raw[K][u], p); }
    template <int J>
    __device__ __forceinline__ C sc() const { return s[J]; }
};

// Operand values of one element, loaded one by one.
template <int DT, int NL, int NS>
struct ElemCtx {
    using C = typename Tr<DT>::C;
    const void *const (&op)[NL];
    const C (&s)[NS];
    int64_t i;
    template <int K>
    __device__ __forceinline__ C ld() const { return Tr<DT>::ld1(op[K], i); }
    template <int J>
    __device__ __forceinline__ C sc() const { return s[J]; }
};

template <class E, int DT, int U, bool NT>
__global__ __launch_bounds__(kBlock) void k_eval_tree(EvalArgs<DT> a) {
    using C = typename Tr<DT>::C;
    constexpr int V = Tr<DT>::V;
    constexpr int NL = E::n_loads > 0 ? E::n_loads : 1;
    constexpr int NS = E::n_scal > 0 ? E::n_scal : 1;
    const void *op[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) op[k] = a.ops[k];
    C s[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) s[j] = a.sc[j];

    constexpr int64_t tile = (int64_t)kBlock * U * V;
    const int64_t n_tiles = a.vec ? a.n / tile : 0;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t c0 = t * (kBlock * U) + threadIdx.x;  // this lane's first chunk
        u32x4 raw[NL][U];
#pragma unroll
        for (int k = 0; k < E::n_loads; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) raw[k][u] = ld16<NT>((const u32x4 *)op[k] + c0 + u * kBlock);
        u32x4 res[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            C r[V];
#pragma unroll
            for (int p = 0; p < V; ++p) r[p] = E::ev(ChunkCtx<DT, NL, U, NS>{raw, s, u, p});
            res[u] = Tr<DT>::template pack<V>(r);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) st16<NT>((u32x4 *)a.out + c0 + u * kBlock, res[u]);
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = n_tiles * tile + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += stride)
        Tr<DT>::st1(a.out, i, E::ev(ElemCtx<DT, NL, NS>{op, s, i}));
}

}  // namespace salt
