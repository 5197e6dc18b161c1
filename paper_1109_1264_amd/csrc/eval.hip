// eval.hip -- fused element-wise evaluation kernels for gfx950.
//
// One kernel pass evaluates a whole expression tree per element (loop
// fusion, Sec. 2): every operand is read once, the result written once, and
// intermediates stay in registers. The loop body follows the paper's
// instruction packages (Sec. 4.3): each lane first issues all of its 16-byte
// loads for a tile (U chunks per operand), then evaluates the tree on the
// loaded registers, then issues all of its stores. U plays the role of the
// paper's number of packages per loop, picked by measurement per tree, type
// and size (Sec. 4.3, last paragraph), and the 16-byte chunk the role of its
// SIMD vector. Elements after the last whole tile, and every element when an
// array is not 16-byte aligned, go through a per-element loop: the paper's
// scalar tail (Listing 2) and its non-specialised fallback.
//
// Two kernel families:
//  * k_eval_tree<E, ...> (eval_tree.hpp): the tree E is a compile-time type
//    (expr.hpp) and the kernel is straight-line code for it (ahead-of-time
//    catalogue here; any other tree compiled at run time by jit.hip).
//  * k_eval_interp<...>: any valid program. The program is uniform across the
//    grid, so its instruction loop runs on the scalar unit; the top of the
//    per-lane stack stays in registers and the rest lives in LDS
//    (interp.hpp).
#include "device.hpp"
#include "eval_tree.hpp"
#include "expr.hpp"
#include "interp.hpp"
#include "launch.hpp"

namespace salt {

// ---------------------------------------------------------------------------
// generic interpreter (interp.hpp)
// ---------------------------------------------------------------------------

template <int DT, int U, bool NT, int NL>
__global__ __launch_bounds__(kBlock) void k_eval_interp(EvalArgs<DT> a, InterpProg g) {
    using C = typename Tr<DT>::C;
    constexpr int V = Tr<DT>::V;
    extern __shared__ __align__(16) unsigned char interp_smem[];
    C *lds = (C *)interp_smem;
    constexpr int64_t tile = (int64_t)kBlock * U * V;
    const int64_t n_tiles = a.vec ? a.n / tile : 0;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t c0 = t * (kBlock * U) + threadIdx.x;
        u32x4 raw[NL][U];
#pragma unroll
        for (int k = 0; k < NL; ++k)
            if (k < g.n_loads)
#pragma unroll
                for (int u = 0; u < U; ++u) raw[k][u] = ld16<NT>((const u32x4 *)a.ops[k] + c0 + u * kBlock);
        C tos[U * V];
        interp_run<U * V, NL>(g, a.sc, [&](int k, int j) { return Tr<DT>::get(raw[k][j / V], j % V); }, tos, lds);
#pragma unroll
        for (int u = 0; u < U; ++u) st16<NT>((u32x4 *)a.out + c0 + u * kBlock, Tr<DT>::template pack<V>(&tos[u * V]));
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = n_tiles * tile + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += stride) {
        C tos[1];
        interp_run<1, NL>(g, a.sc, [&](int k, int) { return Tr<DT>::ld1(a.ops[k], i); }, tos, lds);
        Tr<DT>::st1(a.out, i, tos[0]);
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <int DT>
static EvalArgs<DT> make_args(const EvalLaunch &L) {
    EvalArgs<DT> a;
    for (int k = 0; k < SALT_MAX_OPERANDS; ++k) a.ops[k] = L.ops[k];
    // Scalars are rounded once (nearest-even) to the compute type here.
    for (int j = 0; j < SALT_MAX_SCALARS; ++j) a.sc[j] = (typename Tr<DT>::C)L.sc[j];
    a.out = L.out;
    a.n = L.n;
    a.vec = L.vec;
    return a;
}

int64_t eval_grid(const EvalLaunch &L, int64_t tile) {
    const int64_t n_tiles = L.vec ? L.n / tile : 0;
    int64_t g;
    if (n_tiles > 0) {
        g = L.blocks > 0 ? (L.blocks < n_tiles ? L.blocks : n_tiles) : n_tiles;
    } else {
        g = (L.n + kBlock - 1) / kBlock;
        const int64_t cap = L.blocks > 0 ? L.blocks : 8192;
        if (g > cap) g = cap;
    }
    if (g < 1) g = 1;
    if (g > 0x7fffffff) g = 0x7fffffff;
    return g;
}

template <int DT>
static dim3 grid_for(const EvalLaunch &L, int U) {
    return dim3((unsigned)eval_grid(L, (int64_t)kBlock * U * Tr<DT>::V));
}

template <class E, int DT, int U, bool NT>
static hipError_t launch_tree_u(const EvalLaunch &L) {
    hipLaunchKernelGGL((k_eval_tree<E, DT, U, NT>), grid_for<DT>(L, U), dim3(kBlock), 0,
                       (hipStream_t)L.stream, make_args<DT>(L));
    return hipGetLastError();
}

template <class E, int DT>
static hipError_t launch_tree(const EvalLaunch &L) {
    const bool nt = L.nontemporal != 0;
    switch (L.unroll) {
        case 1: return nt ? launch_tree_u<E, DT, 1, true>(L) : launch_tree_u<E, DT, 1, false>(L);
        case 2: return nt ? launch_tree_u<E, DT, 2, true>(L) : launch_tree_u<E, DT, 2, false>(L);
        case 4: return nt ? launch_tree_u<E, DT, 4, true>(L) : launch_tree_u<E, DT, 4, false>(L);
        case 8: return nt ? launch_tree_u<E, DT, 8, true>(L) : launch_tree_u<E, DT, 8, false>(L);
        default: return hipErrorInvalidValue;
    }
}

template <class E>
static EvalFn tree_fn(int dtype) {
    switch (dtype) {
        case SALT_F64: return &launch_tree<E, SALT_F64>;
        case SALT_F32: return &launch_tree<E, SALT_F32>;
        case SALT_BF16: return &launch_tree<E, SALT_BF16>;
        case SALT_F16: return &launch_tree<E, SALT_F16>;
        default: return nullptr;
    }
}

EvalFn catalogue_launcher(int id, int dtype) {
    switch (id) {
#define SALT_CAT_CASE(name, ...) \
    case cat::id_##name: return tree_fn<cat::name>(dtype);
        SALT_CATALOGUE(SALT_CAT_CASE)
#undef SALT_CAT_CASE
        default: return nullptr;
    }
}

int catalogue_program(int id, uint32_t *tokens, int cap, const char **name) {
    uint32_t buf[SALT_MAX_TOKENS];
    int len = 0;
    switch (id) {
#define SALT_CAT_EMIT(nm, ...)       \
    case cat::id_##nm:               \
        cat::nm::emit(buf, len);     \
        if (name) *name = #nm;       \
        break;
        SALT_CATALOGUE(SALT_CAT_EMIT)
#undef SALT_CAT_EMIT
        default: return -1;
    }
    for (int t = 0; t < len && t < cap; ++t) tokens[t] = buf[t];
    return len;
}

template <int DT, int U, bool NT, int NL>
static hipError_t launch_interp_u(const EvalLaunch &L, const InterpProg &g, int need) {
    const size_t lds = interp_lds_bytes(need, U * Tr<DT>::V, sizeof(typename Tr<DT>::C));
    hipLaunchKernelGGL((k_eval_interp<DT, U, NT, NL>), grid_for<DT>(L, U), dim3(kBlock), lds,
                       (hipStream_t)L.stream, make_args<DT>(L), g);
    return hipGetLastError();
}

template <int DT, int U>
static hipError_t launch_interp_nl(const EvalLaunch &L, const InterpProg &g, int nl, int need) {
    const bool nt = L.nontemporal != 0;
    switch (nl) {
        case 2: return nt ? launch_interp_u<DT, U, true, 2>(L, g, need) : launch_interp_u<DT, U, false, 2>(L, g, need);
        case 4: return nt ? launch_interp_u<DT, U, true, 4>(L, g, need) : launch_interp_u<DT, U, false, 4>(L, g, need);
        default: return nt ? launch_interp_u<DT, U, true, 8>(L, g, need) : launch_interp_u<DT, U, false, 8>(L, g, need);
    }
}

// U, the chunks per lane that one run of the program covers, is the launch
// knob's unroll (1, 2 or 4; 8 runs as 4), lowered until the LDS stack fits;
// NL, the operand registers, is the smallest of 2, 4, 8 covering the
// program.
template <int DT>
static hipError_t launch_interp_dt(const EvalLaunch &L, const InterpProg &g, int nl, int need) {
    const int u = interp_fit_unroll(L.unroll > 4 ? 4 : L.unroll, need, Tr<DT>::V, sizeof(typename Tr<DT>::C));
    if (u >= 4) return launch_interp_nl<DT, 4>(L, g, nl, need);
    if (u == 2) return launch_interp_nl<DT, 2>(L, g, nl, need);
    return launch_interp_nl<DT, 1>(L, g, nl, need);
}

hipError_t launch_interp(const EvalLaunch &L, const Program &p, int dtype) {
    InterpProg g;
    g.clear();
    for (int t = 0; t < p.len; ++t) g.set(t, p.code[t], p.sarg[t]);
    g.len = p.len;
    g.n_loads = p.n_loads;
    const int nl = interp_bound(p.n_loads);
    switch (dtype) {
        case SALT_F64: return launch_interp_dt<SALT_F64>(L, g, nl, p.stack_need);
        case SALT_F32: return launch_interp_dt<SALT_F32>(L, g, nl, p.stack_need);
        case SALT_BF16: return launch_interp_dt<SALT_BF16>(L, g, nl, p.stack_need);
        case SALT_F16: return launch_interp_dt<SALT_F16>(L, g, nl, p.stack_need);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace salt
