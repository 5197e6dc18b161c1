// reduce_tree.hpp -- dot(P, Q) and nrm2(P) for a pair of compile-time trees
// (the lazy evaluation of a tree inside a dot product or a norm, Sec. 2),
// pass 1 of the two-pass scheme of reduce_kernels.hpp.
//
// Device code only: the library instantiates it for its catalogue of
// reduction pairs, and the run-time compiler (jit.hip) for any other pair,
// from this same text, so both give the bits of the interpreted form.
#pragma once

#include "expr.hpp"
#include "reduce_common.hpp"

namespace salt {

// The same reductions for a pair (P, Q) of compile-time trees (or P alone
// for nrm2): straight-line code per element instead of the interpreter.
// Values, roundings, zeros past n and the accumulation order are those of
// k_reduce_expr, so the bits are the same; a single tile stores its result
// from here, as salt_dot does.
template <int DT, int NL, int U, int NS>
struct RChunkCtx {
    using C = typename Tr<DT>::C;
    const u32x4 (&raw)[NL][U];
    const C (&s)[NS];
    int u, p;
    template <int K>
    __device__ __forceinline__ C ld() const { return Tr<DT>::get(raw[K][u], p); }
    template <int J>
    __device__ __forceinline__ C sc() const { return s[J]; }
};

template <int DT>
struct RedTreeArgs {
    const void *ops[SALT_MAX_OPERANDS];  // canonical numbering of the pair
    typename Tr<DT>::C sc[SALT_MAX_SCALARS];
    double *ws;
    int64_t n;
    int32_t vec;
    void *result;
    int32_t final_store;  // n fits one tile: store the result from here
};

template <class P, class Q, int DT, int UR, bool NT>
__global__ __launch_bounds__(kBlock) void k_reduce_tree(RedTreeArgs<DT> a) {
    using C = typename Tr<DT>::C;
    constexpr bool NRM = Q::len == 0;
    constexpr int V = Tr<DT>::V;
    constexpr int64_t T = tile_elems<DT>();
    constexpr int NL = cmax(cmax(P::n_loads, Q::n_loads), 1);
    constexpr int NS = cmax(cmax(P::n_scal, Q::n_scal), 1);
    const int64_t n_tiles = (a.n + T - 1) / T;
    const int64_t n_full = a.vec ? a.n / T : 0;
    __shared__ double lds[kBlock / 64];
    const void *op[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) op[k] = a.ops[k];
    C s[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) s[j] = a.sc[j];
    // the values salt_eval would store, multiplied in the accumulators
    const auto add_chunk = [&](Acc<DT>(&acc)[V], const u32x4(&raw)[NL][UR], int u, int64_t first, bool check) {
#pragma unroll
        for (int p = 0; p < V; ++p) {
            const RChunkCtx<DT, NL, UR, NS> g{raw, s, u, p};
            C x = Tr<DT>::round(P::ev(g));
            C y = x;
            if constexpr (!NRM) y = Tr<DT>::round(Q::ev(g));
            if (check && first + p >= a.n) x = y = (C)0;
            acc[p].add(x, y);
        }
    };
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        Acc<DT> acc[V];
        const int64_t c0 = t * ((int64_t)kBlock * kChunksPerLane) + threadIdx.x;
        if (t < n_full) {
#pragma unroll 1
            for (int it0 = 0; it0 < kChunksPerLane; it0 += UR) {
                u32x4 raw[NL][UR];
#pragma unroll
                for (int k = 0; k < P::n_loads || k < Q::n_loads; ++k)
#pragma unroll
                    for (int u = 0; u < UR; ++u) raw[k][u] = ld16<NT>((const u32x4 *)op[k] + c0 + (int64_t)(it0 + u) * kBlock);
#pragma unroll
                for (int u = 0; u < UR; ++u) add_chunk(acc, raw, u, 0, false);
            }
        } else {
            // the short tile: its rows with elements only, element-wise loads
            // with zeros past n, and the values past n set to zero
            const int64_t m = a.n - t * T;
            const int rows = m < T ? (int)((m + (int64_t)kBlock * V - 1) / ((int64_t)kBlock * V)) : kChunksPerLane;
#pragma unroll 1
            for (int it0 = 0; it0 < rows; it0 += UR) {
                u32x4 raw[NL][UR];
#pragma unroll
                for (int k = 0; k < P::n_loads || k < Q::n_loads; ++k)
#pragma unroll
                    for (int u = 0; u < UR; ++u) {
                        raw[k][u] = u32x4{0u, 0u, 0u, 0u};
                        if (it0 + u < rows)
                            raw[k][u] = load_chunk_guarded<DT, NT>(op[k], c0 + (int64_t)(it0 + u) * kBlock, a.n, a.vec);
                    }
#pragma unroll
                for (int u = 0; u < UR; ++u)
                    if (it0 + u < rows) add_chunk(acc, raw, u, (c0 + (int64_t)(it0 + u) * kBlock) * V, true);
            }
        }
        const double v = block_sum<kBlock / 64>(lane_value<DT>(acc), lds);
        if (threadIdx.x == 0) {
            if (a.final_store) store_result<DT, NRM>(a.result, v);
            else a.ws[t] = v;
        }
    }
}

}  // namespace salt
