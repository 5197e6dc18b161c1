// device.hpp -- element types, 16-byte chunk access and conversions for the
// gfx950 kernels.
//
// Every lane moves data in 16-byte chunks (one global_load_dwordx4 /
// global_store_dwordx4): 2 binary64, 4 binary32 or 8 16-bit values. This is
// the GPU counterpart of the paper's vectorizer class (Sec. 3): the
// expression code is written once against `Tr<DT>` and the element type picks
// the load width and conversions. 16-bit storage is widened exactly to
// binary32 on load and rounded to nearest-even once on store (the hardware
// cvt instructions, default round-to-nearest mode).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "salt.h"

#pragma clang fp contract(off)

namespace salt {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kBlock = 256;  // threads per workgroup (4 waves of 64)

template <int DT>
struct Tr;

template <>
struct Tr<SALT_F64> {
    using S = double;  // stored element
    using C = double;  // compute type
    static constexpr int V = 2;
    __device__ __forceinline__ static C get(const u32x4 &c, int p) {
        return __builtin_bit_cast(f64x2, c)[p];
    }
    template <int N>
    __device__ __forceinline__ static u32x4 pack(const C *v) {
        f64x2 r;
        r[0] = v[0];
        r[1] = v[1];
        return __builtin_bit_cast(u32x4, r);
    }
    __device__ __forceinline__ static C ld1(const void *p, int64_t i) { return ((const S *)p)[i]; }
    __device__ __forceinline__ static void st1(void *p, int64_t i, C v) { ((S *)p)[i] = v; }
    // The value a store would keep (storage equals compute type here).
    __device__ __forceinline__ static C round(C v) { return v; }
};

template <>
struct Tr<SALT_F32> {
    using S = float;
    using C = float;
    static constexpr int V = 4;
    __device__ __forceinline__ static C get(const u32x4 &c, int p) {
        return __builtin_bit_cast(f32x4, c)[p];
    }
    template <int N>
    __device__ __forceinline__ static u32x4 pack(const C *v) {
        f32x4 r;
        r[0] = v[0];
        r[1] = v[1];
        r[2] = v[2];
        r[3] = v[3];
        return __builtin_bit_cast(u32x4, r);
    }
    __device__ __forceinline__ static C ld1(const void *p, int64_t i) { return ((const S *)p)[i]; }
    __device__ __forceinline__ static void st1(void *p, int64_t i, C v) { ((S *)p)[i] = v; }
    __device__ __forceinline__ static C round(C v) { return v; }
};

// bfloat16: the top half of a binary32 pattern.
template <>
struct Tr<SALT_BF16> {
    using S = uint16_t;
    using C = float;
    static constexpr int V = 8;
    __device__ __forceinline__ static C get(const u32x4 &c, int p) {
        const unsigned w = c[p >> 1];
        return __uint_as_float((p & 1) ? (w & 0xffff0000u) : (w << 16));
    }
    __device__ __forceinline__ static unsigned pack2(C lo, C hi) {
        f32x2 f;
        f[0] = lo;
        f[1] = hi;
        return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2));
    }
    template <int N>
    __device__ __forceinline__ static u32x4 pack(const C *v) {
        u32x4 r;
        r[0] = pack2(v[0], v[1]);
        r[1] = pack2(v[2], v[3]);
        r[2] = pack2(v[4], v[5]);
        r[3] = pack2(v[6], v[7]);
        return r;
    }
    __device__ __forceinline__ static C ld1(const void *p, int64_t i) {
        return __uint_as_float((unsigned)((const S *)p)[i] << 16);
    }
    __device__ __forceinline__ static void st1(void *p, int64_t i, C v) {
        ((S *)p)[i] = __builtin_bit_cast(uint16_t, (__bf16)v);
    }
    // The value a store would keep: rounded to bfloat16, widened back.
    __device__ __forceinline__ static C round(C v) {
        return __uint_as_float((unsigned)__builtin_bit_cast(uint16_t, (__bf16)v) << 16);
    }
};

// A binary32 value the compiler must treat as already computed: it cannot
// fold the operation that produced it into what consumes it. The narrowing
// to binary16 needs this: gfx950's mixed-precision fma instructions can
// multiply binary32 operands and round the exact product straight to
// binary16, and the compiler forms them from a multiply followed by the
// conversion (even with contraction off). That rounds once where the
// arithmetic rounds twice (to binary32, then to binary16), and the results
// differ in rare halfway cases. An empty asm statement with the value as
// an in-out register operand costs no instruction.
__device__ __forceinline__ float opaque_f32(float v) {
    asm("" : "+v"(v));
    return v;
}

// binary16.
template <>
struct Tr<SALT_F16> {
    using S = uint16_t;
    using C = float;
    static constexpr int V = 8;
    __device__ __forceinline__ static C get(const u32x4 &c, int p) {
        return (float)__builtin_bit_cast(f16x8, c)[p];
    }
    template <int N>
    __device__ __forceinline__ static u32x4 pack(const C *v) {
        f16x8 r;
#pragma unroll
        for (int p = 0; p < 8; ++p) r[p] = (_Float16)opaque_f32(v[p]);
        return __builtin_bit_cast(u32x4, r);
    }
    __device__ __forceinline__ static C ld1(const void *p, int64_t i) {
        return (float)((const _Float16 *)p)[i];
    }
    __device__ __forceinline__ static void st1(void *p, int64_t i, C v) {
        ((_Float16 *)p)[i] = (_Float16)opaque_f32(v);
    }
    __device__ __forceinline__ static C round(C v) { return (float)(_Float16)opaque_f32(v); }
};

// 16-byte loads and stores, optionally non-temporal (streaming data that is
// not reused should not displace cached data).
template <bool NT>
__device__ __forceinline__ u32x4 ld16(const u32x4 *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st16(u32x4 *p, u32x4 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

}  // namespace salt
