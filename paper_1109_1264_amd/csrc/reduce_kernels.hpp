// reduce_kernels.hpp -- dot and nrm2 (the reductions at the root of an expression
// tree, Sec. 2; the node's reduction step, Sec. 4.2), and asum (the BLAS
// level-1 sum of magnitudes) for gfx950.
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
#pragma once

#include "expr.hpp"
#include "interp.hpp"
#include "launch.hpp"
#include "reduce_common.hpp"
#include "reduce_tree.hpp"

namespace salt {

struct RedArgs {
    const void *x;
    const void *y;
    double *ws;
    int64_t n;
    int32_t vec;
    // A single tile (n <= tile size): the combine of one partial is the
    // partial itself (it is never -0, so adding the zeros of the other lanes
    // keeps its bits), so pass 1 rounds and stores the result directly and
    // pass 2 is not launched.
    void *result;
    int32_t final_store;
};

// The value a reduction adds for element (x, y): x*y (dot), x*x (nrm2), or
// |x|*1 (asum; the product is exact, so the accumulators add |x| itself).
template <int DT, int MODE>
__device__ __forceinline__ void acc_add(Acc<DT> &acc, typename Tr<DT>::C x, typename Tr<DT>::C y) {
    using C = typename Tr<DT>::C;
    if constexpr (MODE == kModeDot) acc.add(x, y);
    else if constexpr (MODE == kModeNrm2) acc.add(x, x);
    else acc.add(x < (C)0 ? -x : x, (C)1);
}

template <int DT, int UR, bool NT, int MODE>
__global__ __launch_bounds__(kBlock) void k_reduce_pass1(RedArgs a) {
    constexpr bool NRM = MODE != kModeDot;  // one operand
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
        // The last tile of aligned arrays: range-checked buffer loads over its
        // whole chunks (zeros past them), and the chunk that straddles the
        // end, if any, element by element by its lane. Same values as the
        // element-wise path, without a branch per chunk.
        const bool ragged = !full && a.vec;
        const int64_t m = a.n - t * T;
        const int32_t whole = ragged ? (int32_t)(m / V) : 0;
        const int32_t straddle = ragged && (m % V) ? whole : -1;
        __amdgpu_buffer_rsrc_t rx, ry;
        if (ragged) {
            rx = rsrc((const typename Tr<DT>::S *)a.x + t * T, whole * 16);
            ry = rsrc((const typename Tr<DT>::S *)(NRM ? a.x : a.y) + t * T, whole * 16);
        }
        const auto accumulate = [&](const u32x4 (&xr)[UR], const u32x4 (&yr)[UR]) {
#pragma unroll
            for (int u = 0; u < UR; ++u)
#pragma unroll
                for (int p = 0; p < V; ++p) {
                    const auto xv = Tr<DT>::get(xr[u], p);
                    acc_add<DT, MODE>(acc[p], xv, NRM ? xv : Tr<DT>::get(yr[u], p));
                }
        };
        if (full) {
#pragma unroll
            for (int it0 = 0; it0 < kChunksPerLane; it0 += UR) {
                u32x4 xr[UR], yr[UR];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    xr[u] = ld16<NT>(x16 + c0 + (int64_t)(it0 + u) * kBlock);
                    if constexpr (!NRM) yr[u] = ld16<NT>(y16 + c0 + (int64_t)(it0 + u) * kBlock);
                }
                accumulate(xr, yr);
            }
        } else {
            // Chunk rows (kBlock chunks each) that hold elements: rows past
            // them would only add the product +0, which leaves an
            // accumulator's bits unchanged (it is never -0), so a short tile
            // neither loads nor adds them. A burst issues all its rows'
            // loads before it adds any.
            const int rows = m < T ? (int)((m + (int64_t)kBlock * V - 1) / ((int64_t)kBlock * V)) : kChunksPerLane;
            const u32x4 zero = {0u, 0u, 0u, 0u};
#pragma unroll 1
            for (int it0 = 0; it0 < rows; it0 += UR) {
                u32x4 xr[UR], yr[UR];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    xr[u] = zero;
                    if constexpr (!NRM) yr[u] = zero;
                    if (it0 + u >= rows) continue;
                    if (ragged) {
                        const int32_t off = ((it0 + u) * kBlock + (int32_t)threadIdx.x) * 16;
                        xr[u] = bld16<NT>(rx, off);
                        if constexpr (!NRM) yr[u] = bld16<NT>(ry, off);
                    } else {
                        const int64_t ci = c0 + (int64_t)(it0 + u) * kBlock;
                        xr[u] = load_chunk_guarded<DT, NT>(a.x, ci, a.n, a.vec);
                        if constexpr (!NRM) yr[u] = load_chunk_guarded<DT, NT>(a.y, ci, a.n, a.vec);
                    }
                }
                if (ragged) {
#pragma unroll
                    for (int u = 0; u < UR; ++u)
                        if (straddle >= 0 && it0 + u == straddle / kBlock && (int)threadIdx.x == straddle % kBlock) {
                            const int64_t ci = c0 + (int64_t)(it0 + u) * kBlock;
                            xr[u] = load_chunk_guarded<DT, NT>(a.x, ci, a.n, false);
                            if constexpr (!NRM) yr[u] = load_chunk_guarded<DT, NT>(a.y, ci, a.n, false);
                        }
                }
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    if (it0 + u >= rows) continue;
#pragma unroll
                    for (int p = 0; p < V; ++p) {
                        const auto xv = Tr<DT>::get(xr[u], p);
                        acc_add<DT, MODE>(acc[p], xv, NRM ? xv : Tr<DT>::get(yr[u], p));
                    }
                }
            }
        }
        const double v = block_sum<kBlock / 64>(lane_value<DT>(acc), lds);
        if (threadIdx.x == 0) {
            if (a.final_store) store_result<DT, MODE == kModeNrm2>(a.result, v);
            else a.ws[t] = v;
        }
    }
}

// dot(P(x...), Q(y...)) and nrm2(P(x...)) in one pass: the operands read by
// either program are loaded once per chunk; P and Q run back to back on one
// interpreter stack (Q's codes shifted up one slot on the host, so P's value
// stays in slot 0, in LDS, and Q's ends on top), and the values enter the
// accumulators in exactly the order of k_reduce_pass1, with elements past n
// set to zero. Each value is first rounded to the storage type, as a store
// would round it (16-bit storage), so the exact-product accumulators stay
// exact. The result therefore has
// the same bits as evaluating P and Q into vectors and calling salt_dot on
// them, without writing or re-reading those vectors (the lazy evaluation of
// a tree inside a dot product or norm).
template <int DT>
struct RedExprArgs {
    const void *ops[SALT_MAX_OPERANDS];  // the caller's operand numbering
    typename Tr<DT>::C sc[SALT_MAX_SCALARS];
    double *ws;
    int64_t n;
    int32_t vec;
    uint32_t mask;  // operands read by either program
};

template <int DT, int UR, bool NT, bool NRM, int NL>
__global__ __launch_bounds__(kBlock) void k_reduce_expr(RedExprArgs<DT> a, InterpProg2 g) {
    using C = typename Tr<DT>::C;
    constexpr int V = Tr<DT>::V;
    constexpr int EL = UR * V;
    constexpr int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (a.n + T - 1) / T;
    const int64_t n_full = a.vec ? a.n / T : 0;
    __shared__ double lds[kBlock / 64];
    extern __shared__ __align__(16) unsigned char interp_smem[];
    C *stack = (C *)interp_smem;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        Acc<DT> acc[V];
        const int64_t c0 = t * ((int64_t)kBlock * kChunksPerLane) + threadIdx.x;
        const bool full = t < n_full;
        // A short tile stops after its last chunk row with data (the rows
        // past it would add +0, which changes no accumulator's bits).
        const int64_t m = a.n - t * T;
        const int rows = m < T ? (int)((m + (int64_t)kBlock * V - 1) / ((int64_t)kBlock * V)) : kChunksPerLane;
        // One burst per iteration, not unrolled: the interpreter loop inside
        // would otherwise be copied per burst.
#pragma unroll 1
        for (int it0 = 0; it0 < rows; it0 += UR) {
            u32x4 raw[NL][UR];
#pragma unroll
            for (int k = 0; k < NL; ++k)
                if ((a.mask >> k) & 1u)
#pragma unroll
                    for (int u = 0; u < UR; ++u) {
                        const int64_t ci = c0 + (int64_t)(it0 + u) * kBlock;
                        raw[k][u] = full ? ld16<NT>((const u32x4 *)a.ops[k] + ci)
                                         : load_chunk_guarded<DT, NT>(a.ops[k], ci, a.n, a.vec);
                    }
            const auto get = [&](int k, int j) { return Tr<DT>::get(raw[k][j / V], j % V); };
            C tos[EL];
            interp_run<EL, NL>(g, a.sc, get, tos, stack);
            C xs[EL], ys[EL];
#pragma unroll
            for (int j = 0; j < EL; ++j) {  // the values salt_eval would store
                // P's value is slot 0: the top for nrm2, LDS row 0 under Q's
                xs[j] = Tr<DT>::round(NRM ? tos[j] : stack[j * kBlock + threadIdx.x]);
                ys[j] = Tr<DT>::round(tos[j]);
            }
            if (__builtin_expect(!full, 0)) {
#pragma unroll
                for (int u = 0; u < UR; ++u)
#pragma unroll
                    for (int p = 0; p < V; ++p)
                        if ((c0 + (int64_t)(it0 + u) * kBlock) * V + p >= a.n) {
                            xs[u * V + p] = (C)0;
                            ys[u * V + p] = (C)0;
                        }
            }
#pragma unroll
            for (int u = 0; u < UR; ++u)
#pragma unroll
                for (int p = 0; p < V; ++p) acc[p].add(xs[u * V + p], NRM ? xs[u * V + p] : ys[u * V + p]);
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

template <int DT, int UR, bool NT, int MODE>
static void launch_pass1(const ReduceLaunch &L, int64_t grid) {
    const int64_t T = tile_elems<DT>();
    const int final_store = (L.passes == 3 && L.n <= T) ? 1 : 0;
    RedArgs a{L.x, L.y, L.ws, L.n, L.vec, L.result, final_store};
    hipLaunchKernelGGL((k_reduce_pass1<DT, UR, NT, MODE>), dim3((unsigned)grid), dim3(kBlock), 0,
                       (hipStream_t)L.stream, a);
}

template <int DT, int MODE>
static void pass1_dispatch(const ReduceLaunch &L, int64_t grid) {
    const bool nt = L.nontemporal != 0;
    switch (L.unroll) {
        case 4: nt ? launch_pass1<DT, 4, true, MODE>(L, grid) : launch_pass1<DT, 4, false, MODE>(L, grid); break;
        case 8: nt ? launch_pass1<DT, 8, true, MODE>(L, grid) : launch_pass1<DT, 8, false, MODE>(L, grid); break;
        case 16: nt ? launch_pass1<DT, 16, true, MODE>(L, grid) : launch_pass1<DT, 16, false, MODE>(L, grid); break;
        default: nt ? launch_pass1<DT, 2, true, MODE>(L, grid) : launch_pass1<DT, 2, false, MODE>(L, grid); break;
    }
}

template <int DT>
static hipError_t launch_reduce_dt(const ReduceLaunch &L) {
    const int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (L.passes & 1) ? (L.n + T - 1) / T : L.n_partials;
    if ((L.passes & 1) && n_tiles > 0) {
        int64_t grid = L.blocks > 0 && L.blocks < n_tiles ? L.blocks : n_tiles;
        if (grid > 0x7fffffff) grid = 0x7fffffff;
        if (L.mode == kModeNrm2) pass1_dispatch<DT, kModeNrm2>(L, grid);
        else if (L.mode == kModeAsum) pass1_dispatch<DT, kModeAsum>(L, grid);
        else pass1_dispatch<DT, kModeDot>(L, grid);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!(L.passes & 2) || ((L.passes & 1) && n_tiles == 1)) return hipSuccess;  // pass 1 stored it
    if (L.mode == kModeNrm2)
        hipLaunchKernelGGL((k_reduce_pass2<DT, true>), dim3(1), dim3(kFinalBlock), 0, (hipStream_t)L.stream,
                           (const double *)L.ws, n_tiles, L.result);
    else
        hipLaunchKernelGGL((k_reduce_pass2<DT, false>), dim3(1), dim3(kFinalBlock), 0, (hipStream_t)L.stream,
                           (const double *)L.ws, n_tiles, L.result);
    return hipGetLastError();
}

// Code of `c` with its stack slot moved up by one. Every code is a base plus
// its slot (program.hpp), so this is c + 1; it stays valid while the program
// never uses slot 7 (stack need <= 7): a push then lands in slot <= 7 and a
// binary operation in slot <= 6.
static uint8_t shift_slot(uint8_t c) { return (uint8_t)(c + 1); }

// P's codes, then Q's shifted by one slot (nullptr Q: P alone).
static inline void fill_pair(InterpProg2 &g, const Program &px, const Program *py) {
    g.clear();
    int len = 0;
    for (int t = 0; t < px.len; ++t, ++len) g.set(len, px.code_raw[t], px.sarg_raw[t]);
    if (py)
        for (int t = 0; t < py->len; ++t, ++len) g.set(len, shift_slot(py->code_raw[t]), py->sarg_raw[t]);
    g.len = len;
    g.n_loads = SALT_MAX_OPERANDS;
}

template <int DT, int UR, bool NT, bool NRM, int NL>
static void launch_expr_k(dim3 gd, size_t lds, hipStream_t s, const RedExprArgs<DT> &a, const InterpProg2 &g) {
    hipLaunchKernelGGL((k_reduce_expr<DT, UR, NT, NRM, NL>), gd, dim3(kBlock), lds, s, a, g);
}

template <int DT, int UR, bool NT, bool NRM>
static void launch_expr_l(dim3 gd, size_t lds, hipStream_t s, const RedExprArgs<DT> &a, const InterpProg2 &g,
                          int nl) {
    switch (nl) {
        case 2: launch_expr_k<DT, UR, NT, NRM, 2>(gd, lds, s, a, g); break;
        case 4: launch_expr_k<DT, UR, NT, NRM, 4>(gd, lds, s, a, g); break;
        default: launch_expr_k<DT, UR, NT, NRM, 8>(gd, lds, s, a, g); break;
    }
}

template <int DT, int UR>
static void launch_expr_u(dim3 gd, size_t lds, hipStream_t s, const RedExprArgs<DT> &a, const InterpProg2 &g,
                          int nl, bool nt, bool nrm) {
    if (nrm) {
        if (nt) launch_expr_l<DT, UR, true, true>(gd, lds, s, a, g, nl);
        else launch_expr_l<DT, UR, false, true>(gd, lds, s, a, g, nl);
    } else {
        if (nt) launch_expr_l<DT, UR, true, false>(gd, lds, s, a, g, nl);
        else launch_expr_l<DT, UR, false, false>(gd, lds, s, a, g, nl);
    }
}

// Chunks per lane per interpreter run of the expression reductions: the
// launch knob's unroll (2, 4 or 8), lowered until the LDS stack fits, so
// that one pass of the program covers UR*V values per lane; more chunks
// amortise the program's serial token chain, at the cost of LDS.
template <int DT>
static hipError_t launch_reduce_expr_dt(const ReduceExprLaunch &L, const Program &px, const Program *py) {
    const int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (L.n + T - 1) / T;
    if (n_tiles > 0) {
        RedExprArgs<DT> a;
        for (int k = 0; k < SALT_MAX_OPERANDS; ++k) a.ops[k] = L.ops[k];
        for (int j = 0; j < SALT_MAX_SCALARS; ++j) a.sc[j] = (typename Tr<DT>::C)L.sc[j];
        a.ws = L.ws;
        a.n = L.n;
        a.vec = L.vec;
        a.mask = L.mask;
        InterpProg2 g;
        fill_pair(g, px, py);
        int top = 0;  // highest operand number read, plus one
        for (int k = 0; k < SALT_MAX_OPERANDS; ++k)
            if ((L.mask >> k) & 1u) top = k + 1;
        const int need = py && py->stack_need + 1 > px.stack_need ? py->stack_need + 1 : px.stack_need;
        const int nl = interp_bound(top);
        const int ur = interp_fit_unroll(L.unroll, need, Tr<DT>::V, sizeof(typename Tr<DT>::C));
        const size_t lds = interp_lds_bytes(need, ur * Tr<DT>::V, sizeof(typename Tr<DT>::C));
        int64_t grid = L.blocks > 0 && L.blocks < n_tiles ? L.blocks : n_tiles;
        if (grid > 0x7fffffff) grid = 0x7fffffff;
        const dim3 gd((unsigned)grid);
        hipStream_t s = (hipStream_t)L.stream;
        const bool nt = L.nontemporal != 0, nrm = L.nrm2 != 0;
        if (ur == 8) launch_expr_u<DT, 8>(gd, lds, s, a, g, nl, nt, nrm);
        else if (ur == 4) launch_expr_u<DT, 4>(gd, lds, s, a, g, nl, nt, nrm);
        else if (ur == 2) launch_expr_u<DT, 2>(gd, lds, s, a, g, nl, nt, nrm);
        else launch_expr_u<DT, 1>(gd, lds, s, a, g, nl, nt, nrm);
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

template <class P, class Q, int DT, int UR, bool NT>
static void launch_tree_k(dim3 gd, hipStream_t s, const RedTreeArgs<DT> &a) {
    hipLaunchKernelGGL((k_reduce_tree<P, Q, DT, UR, NT>), gd, dim3(kBlock), 0, s, a);
}

template <class P, class Q, int DT>
static hipError_t launch_reduce_tree_pq(const ReduceExprLaunch &L) {
    constexpr bool NRM = Q::len == 0;
    const int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (L.n + T - 1) / T;
    if (n_tiles == 0) {
        // an empty reduction: pass 2 over no partials stores zero
        hipLaunchKernelGGL((k_reduce_pass2<DT, NRM>), dim3(1), dim3(kFinalBlock), 0, (hipStream_t)L.stream,
                           (const double *)L.ws, (int64_t)0, L.result);
        return hipGetLastError();
    }
    RedTreeArgs<DT> a;
    for (int k = 0; k < SALT_MAX_OPERANDS; ++k) a.ops[k] = L.ops[k];
    for (int j = 0; j < SALT_MAX_SCALARS; ++j) a.sc[j] = (typename Tr<DT>::C)L.sc[j];
    a.ws = L.ws;
    a.n = L.n;
    a.vec = L.vec;
    a.result = L.result;
    a.final_store = n_tiles == 1 ? 1 : 0;
    int64_t grid = L.blocks > 0 && L.blocks < n_tiles ? L.blocks : n_tiles;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    const dim3 gd((unsigned)grid);
    hipStream_t s = (hipStream_t)L.stream;
    const bool nt = L.nontemporal != 0;
    switch (L.unroll) {
        case 2: nt ? launch_tree_k<P, Q, DT, 2, true>(gd, s, a) : launch_tree_k<P, Q, DT, 2, false>(gd, s, a); break;
        case 4: nt ? launch_tree_k<P, Q, DT, 4, true>(gd, s, a) : launch_tree_k<P, Q, DT, 4, false>(gd, s, a); break;
        case 16: nt ? launch_tree_k<P, Q, DT, 16, true>(gd, s, a) : launch_tree_k<P, Q, DT, 16, false>(gd, s, a); break;
        default: nt ? launch_tree_k<P, Q, DT, 8, true>(gd, s, a) : launch_tree_k<P, Q, DT, 8, false>(gd, s, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_tiles == 1) return e;
    hipLaunchKernelGGL((k_reduce_pass2<DT, NRM>), dim3(1), dim3(kFinalBlock), 0, s, (const double *)L.ws, n_tiles,
                       L.result);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_reduce_tree_dt(const ReduceExprLaunch &L, int id) {
    switch (id) {
#define SALT_RCAT_CASE(name) \
    case rcat::id_##name: return launch_reduce_tree_pq<rcat::name::P, rcat::name::Q, DT>(L);
        SALT_RCATALOGUE(SALT_RCAT_CASE)
#undef SALT_RCAT_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_f64(const ReduceLaunch &L);
hipError_t launch_reduce_f32(const ReduceLaunch &L);
hipError_t launch_reduce_bf16(const ReduceLaunch &L);
hipError_t launch_reduce_f16(const ReduceLaunch &L);
hipError_t launch_reduce_expr_f64(const ReduceExprLaunch &L, const Program &px, const Program *py);
hipError_t launch_reduce_expr_f32(const ReduceExprLaunch &L, const Program &px, const Program *py);
hipError_t launch_reduce_expr_bf16(const ReduceExprLaunch &L, const Program &px, const Program *py);
hipError_t launch_reduce_expr_f16(const ReduceExprLaunch &L, const Program &px, const Program *py);
hipError_t launch_reduce_tree_f64(const ReduceExprLaunch &L, int id);
hipError_t launch_reduce_tree_f32(const ReduceExprLaunch &L, int id);
hipError_t launch_reduce_tree_bf16(const ReduceExprLaunch &L, int id);
hipError_t launch_reduce_tree_f16(const ReduceExprLaunch &L, int id);

}  // namespace salt
