// batch_kernels.hpp -- host launchers of the batched kernels
// (batch_device.hpp) for the catalogue trees, by element type.
#pragma once

#include "batch_device.hpp"

namespace salt {

// The per-item combine of the dots' partials (one wave per item).
template <int DT>
static int launch_combine(const BatchLaunch &L) {
    if (L.count == 0) return (int)hipSuccess;
    const int waves = kBlock / 64;
    const int cgrid = (L.count + waves - 1) / waves < 4096 ? (L.count + waves - 1) / waves : 4096;
    hipLaunchKernelGGL((k_batch_combine<DT>), dim3(cgrid), dim3(kBlock), 0, (hipStream_t)L.stream,
                       L.items, L.count, (const double *)L.ws);
    return (int)hipGetLastError();
}

template <class E, int DT, int UR, bool NT, bool DOT>
static int launch_batch_u(const BatchLaunch &L) {
    int64_t grid = L.blocks > 0 && L.blocks < L.total_tiles ? L.blocks : L.total_tiles;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    if (grid > 0)
        hipLaunchKernelGGL((k_batch<E, DT, UR, NT, DOT>), dim3((unsigned)grid), dim3(kBlock), 0,
                           (hipStream_t)L.stream, L.items, L.tiles, L.total_tiles, L.ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !DOT || !L.combine) return (int)e;
    return launch_combine<DT>(L);
}

template <class E, int DT, bool DOT>
static int launch_batch_dot(const BatchLaunch &L) {
    const bool nt = L.nontemporal != 0;
    switch (L.unroll) {
        case 2: return nt ? launch_batch_u<E, DT, 2, true, DOT>(L) : launch_batch_u<E, DT, 2, false, DOT>(L);
        case 4: return nt ? launch_batch_u<E, DT, 4, true, DOT>(L) : launch_batch_u<E, DT, 4, false, DOT>(L);
        case 8: return nt ? launch_batch_u<E, DT, 8, true, DOT>(L) : launch_batch_u<E, DT, 8, false, DOT>(L);
        default: return (int)hipErrorInvalidValue;
    }
}

template <class E, int DT>
static int launch_batch(const BatchLaunch &L) {
    if constexpr (E::n_loads >= 2) {
        if (L.any_dot) return launch_batch_dot<E, DT, true>(L);
    } else {
        if (L.any_dot) return (int)hipErrorInvalidValue;
    }
    return launch_batch_dot<E, DT, false>(L);
}

template <int DT, int UR, bool NT>
static int launch_multi_u(const BatchLaunch &L) {
    int64_t grid = L.blocks > 0 && L.blocks < L.total_tiles ? L.blocks : L.total_tiles;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    if (grid > 0)
        hipLaunchKernelGGL((k_batch_multi<DT, UR, NT>), dim3((unsigned)grid), dim3(kBlock), 0,
                           (hipStream_t)L.stream, L.items, L.tiles, L.total_tiles);
    return (int)hipGetLastError();
}

// Mixed-tree launch: 2 or 4 chunks per burst (8 runs as 4: the six-operand
// tree at 8 would need about 200 registers for its operand chunks alone).
template <int DT>
static int launch_batch_multi(const BatchLaunch &L) {
    if (L.any_dot) return (int)hipErrorInvalidValue;
    const bool nt = L.nontemporal != 0;
    if (L.unroll == 2) return nt ? launch_multi_u<DT, 2, true>(L) : launch_multi_u<DT, 2, false>(L);
    if (L.unroll == 4 || L.unroll == 8) return nt ? launch_multi_u<DT, 4, true>(L) : launch_multi_u<DT, 4, false>(L);
    return (int)hipErrorInvalidValue;
}

// Launcher for catalogue tree `id` in element type DT (instantiated once per
// type, in batch_<type>.hip).
template <int DT>
BatchFn batch_launcher_for(int id) {
    switch (id) {
#define SALT_CAT_CASE(name, ...) \
    case cat::id_##name: return &launch_batch<cat::name, DT>;
        SALT_CATALOGUE(SALT_CAT_CASE)
#undef SALT_CAT_CASE
        default: return nullptr;
    }
}

BatchFn batch_launcher_f64(int id);
BatchFn batch_launcher_f32(int id);
BatchFn batch_launcher_bf16(int id);
BatchFn batch_launcher_f16(int id);
BatchFn batch_multi_launcher_f64();
BatchFn batch_multi_launcher_f32();
BatchFn batch_multi_launcher_bf16();
BatchFn batch_multi_launcher_f16();
BatchFn batch_combine_launcher_f64();
BatchFn batch_combine_launcher_f32();
BatchFn batch_combine_launcher_bf16();
BatchFn batch_combine_launcher_f16();

}  // namespace salt
