// reduce.hip -- dot and nrm2 (the reductions at the root of an expression
// tree, Sec. 2; the node's reduction step, Sec. 4.2) for gfx950.
//
// Deterministic two-pass scheme; the summation order (reduce_common.hpp)
// depends only on n and the element type:
//  pass 1: each tile's binary64 partial goes to ws[tile]. One workgroup per
//          tile, or a grid-stride loop over tiles (which changes nothing
//          inside a tile). Inside a tile each lane loads its 16 chunks in
//          bursts of UR chunks per operand, then accumulates them.
//  pass 2: one workgroup of 1024 lanes combines the partials, takes the square root for
//          nrm2, rounds once to the result type and stores it.
// A tile that runs past n, and every tile of an unaligned call, load chunk by
// chunk with zeros past the end, in the same order: the bits depend neither
// on alignment nor on the launch shape.
#include "launch.hpp"
#include "reduce_common.hpp"

namespace salt {

struct RedArgs {
    const void *x;
    const void *y;
    double *ws;
    int64_t n;
    int32_t vec;
};

template <int DT, int UR, bool NT, bool NRM>
__global__ __launch_bounds__(kBlock) void k_reduce_pass1(RedArgs a) {
    constexpr int V = Tr<DT>::V;
    constexpr int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (a.n + T - 1) / T;
    const int64_t n_full = a.vec ? a.n / T : 0;
    __shared__ double lds[kBlock / 64];
    const u32x4 *x16 = (const u32x4 *)a.x;
    const u32x4 *y16 = (const u32x4 *)(NRM ? a.x : a.y);
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        Acc<DT> acc[V];
        const int64_t c0 = t * ((int64_t)kBlock * kChunksPerLane) + threadIdx.x;
        const bool full = t < n_full;
#pragma unroll
        for (int it0 = 0; it0 < kChunksPerLane; it0 += UR) {
            u32x4 xr[UR], yr[UR];
            if (full) {
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    xr[u] = ld16<NT>(x16 + c0 + (int64_t)(it0 + u) * kBlock);
                    if constexpr (!NRM) yr[u] = ld16<NT>(y16 + c0 + (int64_t)(it0 + u) * kBlock);
                }
            } else {
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    const int64_t ci = c0 + (int64_t)(it0 + u) * kBlock;
                    xr[u] = load_chunk_guarded<DT, NT>(a.x, ci, a.n, a.vec);
                    if constexpr (!NRM) yr[u] = load_chunk_guarded<DT, NT>(a.y, ci, a.n, a.vec);
                }
            }
#pragma unroll
            for (int u = 0; u < UR; ++u)
#pragma unroll
                for (int p = 0; p < V; ++p) {
                    const auto xv = Tr<DT>::get(xr[u], p);
                    acc[p].add(xv, NRM ? xv : Tr<DT>::get(yr[u], p));
                }
        }
        const double v = block_sum<kBlock / 64>(lane_value<DT>(acc), lds);
        if (threadIdx.x == 0) a.ws[t] = v;
    }
}

template <int DT, bool NRM>
__global__ __launch_bounds__(kFinalBlock) void k_reduce_pass2(const double *ws, int64_t n_tiles, void *result) {
    __shared__ double lds[kFinalBlock / 64];
    const double r = combine_partials(ws, n_tiles, lds);
    if (threadIdx.x == 0) store_result<DT, NRM>(result, r);
}

int64_t reduce_tile_elems(int dtype) {
    switch (dtype) {
        case SALT_F64: return tile_elems<SALT_F64>();
        case SALT_F32: return tile_elems<SALT_F32>();
        case SALT_BF16: return tile_elems<SALT_BF16>();
        case SALT_F16: return tile_elems<SALT_F16>();
        default: return 0;
    }
}

template <int DT, int UR, bool NT, bool NRM>
static void launch_pass1(const ReduceLaunch &L, int64_t grid) {
    RedArgs a{L.x, L.y, L.ws, L.n, L.vec};
    hipLaunchKernelGGL((k_reduce_pass1<DT, UR, NT, NRM>), dim3((unsigned)grid), dim3(kBlock), 0,
                       (hipStream_t)L.stream, a);
}

template <int DT, bool NRM>
static void pass1_dispatch(const ReduceLaunch &L, int64_t grid) {
    const bool nt = L.nontemporal != 0;
    switch (L.unroll) {
        case 4: nt ? launch_pass1<DT, 4, true, NRM>(L, grid) : launch_pass1<DT, 4, false, NRM>(L, grid); break;
        case 8: nt ? launch_pass1<DT, 8, true, NRM>(L, grid) : launch_pass1<DT, 8, false, NRM>(L, grid); break;
        case 16: nt ? launch_pass1<DT, 16, true, NRM>(L, grid) : launch_pass1<DT, 16, false, NRM>(L, grid); break;
        default: nt ? launch_pass1<DT, 2, true, NRM>(L, grid) : launch_pass1<DT, 2, false, NRM>(L, grid); break;
    }
}

template <int DT>
static hipError_t launch_reduce_dt(const ReduceLaunch &L) {
    const int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (L.n + T - 1) / T;
    if (n_tiles > 0) {
        int64_t grid = L.blocks > 0 && L.blocks < n_tiles ? L.blocks : n_tiles;
        if (grid > 0x7fffffff) grid = 0x7fffffff;
        if (L.nrm2) pass1_dispatch<DT, true>(L, grid);
        else pass1_dispatch<DT, false>(L, grid);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (L.nrm2)
        hipLaunchKernelGGL((k_reduce_pass2<DT, true>), dim3(1), dim3(kFinalBlock), 0, (hipStream_t)L.stream,
                           (const double *)L.ws, n_tiles, L.result);
    else
        hipLaunchKernelGGL((k_reduce_pass2<DT, false>), dim3(1), dim3(kFinalBlock), 0, (hipStream_t)L.stream,
                           (const double *)L.ws, n_tiles, L.result);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceLaunch &L, int dtype) {
    switch (dtype) {
        case SALT_F64: return launch_reduce_dt<SALT_F64>(L);
        case SALT_F32: return launch_reduce_dt<SALT_F32>(L);
        case SALT_BF16: return launch_reduce_dt<SALT_BF16>(L);
        case SALT_F16: return launch_reduce_dt<SALT_F16>(L);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace salt
