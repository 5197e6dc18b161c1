// reduce_common.hpp -- the fixed summation order shared by salt_dot,
// salt_nrm2 and the batched kernel, so a dot product gives the same bits
// alone and inside a batch.
//
// Tile: T = 256 lanes x 16 chunks x V elements (64 KiB per operand).
//  - lane l takes chunks l, l+256, ..., l+15*256 of the tile in that order;
//    element p of a chunk goes to accumulator slot p;
//  - the slots are combined in binary64 in slot order;
//  - the 64 lanes of a wave are summed by a fixed xor butterfly (both
//    partners add the same two values, so all lanes end with the same bits);
//  - the 4 wave sums are added as (w0 + w1) + (w2 + w3).
// Final combine of P tile partials (one 1024-lane workgroup): lane l sums
// partials l, l+1024, ... in order; the same butterfly; a pairwise tree over
// the 16 wave sums.
// Accumulators: binary64 fused multiply-add for binary64 storage;
// compensated binary32 otherwise (TwoProduct with one fma for binary32
// inputs, exact products for 16-bit inputs, TwoSum for every addition).
#pragma once

#include "device.hpp"

#pragma clang fp contract(off)

namespace salt {

constexpr int kChunksPerLane = 16;

template <int DT>
constexpr int64_t tile_elems() { return (int64_t)kBlock * kChunksPerLane * Tr<DT>::V; }

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
        const float pe = __builtin_fmaf(x, y, -p);  // exact error of the product
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
        // The product of two binary16 values is exact in binary32 (11 + 11
        // significant bits, exponents well inside binary32's range). A
        // bfloat16 product (8 + 8 bits) is exact only while its magnitude
        // lies in binary32's normal range: bfloat16 shares binary32's
        // exponents, so a product below 2^-126 is rounded (to zero below
        // 2^-149) and one above the largest binary32 overflows. Outside
        // that range the result misses the stated error bound.
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

// Sum one value per lane over a workgroup of W waves in the fixed order:
// butterfly inside each wave, then a pairwise tree over the wave sums
// ((w0 + w1) + (w2 + w3) for W = 4). Every thread returns the same value.
// `lds` holds W doubles; ends with a barrier, so `lds` may be reused.
template <int W>
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double w[W];
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = lds[k];
#pragma unroll
    for (int h = W / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int k = 0; k < h; ++k) w[k] = w[2 * k] + w[2 * k + 1];
    __syncthreads();
    return w[0];
}

template <int DT>
__device__ __forceinline__ double lane_value(const Acc<DT> (&acc)[Tr<DT>::V]) {
    double v = acc[0].value();
#pragma unroll
    for (int p = 1; p < Tr<DT>::V; ++p) v = v + acc[p].value();
    return v;
}

// Chunk `ci` (global chunk index) of an array of n elements: a 16-byte load
// when it lies wholly inside and the array is aligned, else element by
// element with zeros past the end.
template <int DT, bool NT>
__device__ __forceinline__ u32x4 load_chunk_guarded(const void *p, int64_t ci, int64_t n, bool vec) {
    constexpr int V = Tr<DT>::V;
    if (vec && (ci + 1) * V <= n) return ld16<NT>((const u32x4 *)p + ci);
    typename Tr<DT>::C v[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
        const int64_t i = ci * V + q;
        v[q] = i < n ? Tr<DT>::ld1(p, i) : (typename Tr<DT>::C)0;
    }
    return Tr<DT>::template pack<V>(v);
}

// Raw buffer resource over `bytes` bytes from p (stride 0; the last word is
// the gfx9-family data-format field). The hardware checks every access
// against the size: loads past it return zero and stores past it are dropped,
// so a ragged tile needs no per-chunk branches.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
template <bool NT>
__device__ __forceinline__ u32x4 bld16(__amdgpu_buffer_rsrc_t r, int32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, NT ? 2 : 0);
}
template <bool NT>
__device__ __forceinline__ void bst16(__amdgpu_buffer_rsrc_t r, int32_t off, u32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, NT ? 2 : 0);
}

// Final combine over `count` partials by one workgroup of kFinalBlock lanes:
// lane l adds partials l, l + 1024, l + 2048, ... in that order, then
// block_sum. The value is returned in every thread. Loads are issued 32 at a
// time (one round trip for up to 32768 partials, i.e. 2^28 binary64
// elements); slots past `count` add +0, which leaves the sum's bits
// unchanged (it starts at +0 and is never -0).
constexpr int kFinalBlock = 1024;

__device__ __forceinline__ double combine_partials(const double *part, int64_t count, double *lds) {
    constexpr int kBurst = 32;
    double v = 0.0;
    for (int64_t base = threadIdx.x; base < count; base += (int64_t)kBurst * kFinalBlock) {
        double q[kBurst];
#pragma unroll
        for (int j = 0; j < kBurst; ++j) {
            const int64_t i = base + (int64_t)j * kFinalBlock;
            q[j] = i < count ? part[i] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kBurst; ++j) v = v + q[j];
    }
    return block_sum<kFinalBlock / 64>(v, lds);
}

// The same arithmetic as combine_partials, done by a single wave: lane j of
// virtual wave v plays lane 64v + j of the 1024-lane combine, the 16 virtual
// waves' sums go through the same pairwise tree, so the result has the same
// bits. Used where one workgroup per reduction would be wasteful (many small
// reductions). Each pass over 1024 partials issues its 16 loads together;
// slots past `count` add +0, and a virtual wave with no partial sums to +0
// without being visited: adding +0 leaves any sum that is not -0 unchanged,
// and these sums never are -0 (they start at +0).
__device__ __forceinline__ double combine_partials_wave(const double *part, int64_t count) {
    constexpr int W = kFinalBlock / 64;
    const int lane = threadIdx.x & 63;
    double v[W];
#pragma unroll
    for (int vw = 0; vw < W; ++vw) v[vw] = 0.0;
    for (int64_t base = 0; base < count; base += kFinalBlock) {
        double q[W];
#pragma unroll
        for (int vw = 0; vw < W; ++vw) {
            const int64_t i = base + vw * 64 + lane;
            q[vw] = i < count ? part[i] : 0.0;
        }
#pragma unroll
        for (int vw = 0; vw < W; ++vw) v[vw] = v[vw] + q[vw];
    }
    double w[W];
#pragma unroll
    for (int vw = 0; vw < W; ++vw) w[vw] = (int64_t)vw * 64 < count ? wave_sum(v[vw]) : 0.0;
#pragma unroll
    for (int h = W / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int k = 0; k < h; ++k) w[k] = w[2 * k] + w[2 * k + 1];
    return w[0];
}

template <int DT, bool NRM>
__device__ __forceinline__ void store_result(void *result, double r) {
    if constexpr (NRM) r = __builtin_sqrt(r);
    if constexpr (DT == SALT_F64) *(double *)result = r;
    else *(float *)result = (float)r;
}

}  // namespace salt
