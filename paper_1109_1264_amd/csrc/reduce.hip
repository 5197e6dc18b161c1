// reduce.hip -- dot and nrm2 (the reductions at the root of an expression
// tree, Sec. 2; the node's reduction step, Sec. 4.2) for gfx950.
//
// Deterministic two-pass scheme. The input is cut into fixed tiles of
// T = 256 lanes x 16 chunks x V elements (64 KiB per operand per tile). The
// summation order depends only on (n, dtype):
//  pass 1, one workgroup per tile (or a grid-stride loop over tiles, which
//    changes nothing in a tile):
//    - lane l of the tile takes chunks l, l+256, ..., l+15*256 in that order;
//      element p of each chunk goes to accumulator slot p;
//    - slots are combined in binary64 in slot order;
//    - the 64 lanes of a wave are summed by a fixed xor butterfly (each
//      partner adds the same two values, so every lane holds the same bits);
//    - the 4 wave sums are added as (w0 + w1) + (w2 + w3) and written as the
//      tile's binary64 partial.
//  pass 2, one workgroup: lane l sums partials l, l+1024, ... in order,
//    then the same butterfly and a fixed tree over the 16 waves; nrm2 takes
//    the square root; the value is rounded once to the result type.
// Accumulators: binary64 storage uses binary64 fused multiply-adds. binary32
// storage uses compensated binary32: each product is split exactly into value
// and error with one fma (TwoProduct), each addition into sum and error with
// TwoSum (Knuth), and the errors are summed alongside. 16-bit storage needs
// no TwoProduct: the product of two 8- or 11-bit significands is exact in
// binary32. Lane values go to binary64 before any cross-lane step.
// Elements past n (partial last tile) and every element of an unaligned call
// are read one by one, in the same order, with zeros past the end: the bits
// do not depend on alignment or launch shape.
#include "device.hpp"
#include "launch.hpp"

namespace salt {

constexpr int kChunksPerLane = 16;

template <int DT>
struct Acc;

template <>
struct Acc<SALT_F64> {
    double s = 0.0;
    __device__ __forceinline__ void add(double x, double y) { s = __builtin_fma(x, y, s); }
    __device__ __forceinline__ double value() const { return s; }
};

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float z = s - a;
    e = (a - (s - z)) + (b - z);
}

template <>
struct Acc<SALT_F32> {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x, float y) {
        const float p = x * y;
        const float pe = __builtin_fmaf(x, y, -p);
        float e;
        two_sum(s, p, s, e);
        c = c + (e + pe);
    }
    __device__ __forceinline__ double value() const { return (double)s + (double)c; }
};

struct AccExactProduct {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x, float y) {
        float e;
        two_sum(s, x * y, s, e);
        c = c + e;
    }
    __device__ __forceinline__ double value() const { return (double)s + (double)c; }
};
template <> struct Acc<SALT_BF16> : AccExactProduct {};
template <> struct Acc<SALT_F16> : AccExactProduct {};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

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
    constexpr int64_t T = (int64_t)kBlock * kChunksPerLane * V;
    const int64_t n_tiles = (a.n + T - 1) / T;
    const int64_t n_full = a.vec ? a.n / T : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double wsum[kBlock / 64];
    const u32x4 *x16 = (const u32x4 *)a.x;
    const u32x4 *y16 = (const u32x4 *)(NRM ? a.x : a.y);
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        Acc<DT> acc[V];
        const int64_t c0 = t * ((int64_t)kBlock * kChunksPerLane) + threadIdx.x;
        if (t < n_full) {
#pragma unroll
            for (int it0 = 0; it0 < kChunksPerLane; it0 += UR) {
                u32x4 xr[UR], yr[UR];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    xr[u] = ld16<NT>(x16 + c0 + (int64_t)(it0 + u) * kBlock);
                    if constexpr (!NRM) yr[u] = ld16<NT>(y16 + c0 + (int64_t)(it0 + u) * kBlock);
                }
#pragma unroll
                for (int u = 0; u < UR; ++u)
#pragma unroll
                    for (int p = 0; p < V; ++p) {
                        const auto xv = Tr<DT>::get(xr[u], p);
                        const auto yv = NRM ? xv : Tr<DT>::get(yr[u], p);
                        acc[p].add(xv, yv);
                    }
            }
        } else {
            const void *yp = NRM ? a.x : a.y;
            for (int it = 0; it < kChunksPerLane; ++it) {
                const int64_t e0 = (c0 + (int64_t)it * kBlock) * V;
#pragma unroll
                for (int p = 0; p < V; ++p) {
                    const int64_t i = e0 + p;
                    typename Tr<DT>::C xv = 0, yv = 0;
                    if (i < a.n) {
                        xv = Tr<DT>::ld1(a.x, i);
                        yv = NRM ? xv : Tr<DT>::ld1(yp, i);
                    }
                    acc[p].add(xv, yv);
                }
            }
        }
        double v = acc[0].value();
#pragma unroll
        for (int p = 1; p < V; ++p) v = v + acc[p].value();
        v = wave_sum(v);
        if (lane == 0) wsum[wave] = v;
        __syncthreads();
        if (threadIdx.x == 0) a.ws[t] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
        __syncthreads();
    }
}

constexpr int kFinalBlock = 1024;

template <int DT, bool NRM>
__global__ __launch_bounds__(kFinalBlock) void k_reduce_pass2(const double *ws, int64_t n_tiles, void *result) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n_tiles; i += kFinalBlock) v = v + ws[i];
    v = wave_sum(v);
    __shared__ double wsum[kFinalBlock / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double w[kFinalBlock / 64];
#pragma unroll
        for (int k = 0; k < kFinalBlock / 64; ++k) w[k] = wsum[k];
#pragma unroll
        for (int h = kFinalBlock / 128; h >= 1; h >>= 1)
#pragma unroll
            for (int k = 0; k < h; ++k) w[k] = w[2 * k] + w[2 * k + 1];
        double r = w[0];
        if constexpr (NRM) r = __builtin_sqrt(r);
        if constexpr (DT == SALT_F64) *(double *)result = r;
        else *(float *)result = (float)r;
    }
}

int64_t reduce_tile_elems(int dtype) {
    switch (dtype) {
        case SALT_F64: return (int64_t)kBlock * kChunksPerLane * Tr<SALT_F64>::V;
        case SALT_F32: return (int64_t)kBlock * kChunksPerLane * Tr<SALT_F32>::V;
        case SALT_BF16: return (int64_t)kBlock * kChunksPerLane * Tr<SALT_BF16>::V;
        case SALT_F16: return (int64_t)kBlock * kChunksPerLane * Tr<SALT_F16>::V;
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
    const int64_t T = reduce_tile_elems(DT);
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
        hipLaunchKernelGGL((k_reduce_pass2<DT, true>), dim3(1), dim3(kFinalBlock), 0,
                           (hipStream_t)L.stream, (const double *)L.ws, n_tiles, L.result);
    else
        hipLaunchKernelGGL((k_reduce_pass2<DT, false>), dim3(1), dim3(kFinalBlock), 0,
                           (hipStream_t)L.stream, (const double *)L.ws, n_tiles, L.result);
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
