// interp.hpp -- the per-lane stack machine behind the generic kernels.
//
// A program reaches the kernel as instruction codes (program.hpp): each code
// is a base plus the stack slot it writes -- LOAD k into slot s is 8k + s,
// SCALAR into slot s is 64 + s, ADD/SUB/MUL with the left operand in slot s
// is 72/80/88 + s. The program is the same for every lane, so the decode and
// the switch run on the scalar unit (readfirstlane says so to the compiler).
//
// The top of the stack lives in registers (EL values per lane); the slots
// below it live in LDS, one row of 256 lanes per (slot, value), so a push
// writes the old top to LDS and a binary operation reads its left operand
// from LDS: one LDS access per token, conflict-free (consecutive lanes,
// consecutive addresses). Registers hold only the operands' loaded chunks and
// the top of stack, whatever the program's depth.
#pragma once

#include "device.hpp"

namespace salt {

// A program as instruction codes; CAP tokens (one program, or two run back
// to back by the expression reductions). Codes are packed four to a 32-bit
// word: a dynamically indexed byte of a kernel argument can only be fetched
// by a vector memory load (one memory round trip per token), a dword by the
// scalar unit from its cache.
template <int CAP>
struct InterpCodes {
    uint32_t code[CAP / 4];
    uint32_t sarg[CAP / 4];
    int32_t len;
    int32_t n_loads;
    __host__ void set(int t, uint8_t c, uint8_t a) {
        const int sh = (t & 3) * 8;
        code[t >> 2] = (code[t >> 2] & ~(0xffu << sh)) | ((uint32_t)c << sh);
        sarg[t >> 2] = (sarg[t >> 2] & ~(0xffu << sh)) | ((uint32_t)a << sh);
    }
    __host__ void clear() {
        for (int w = 0; w < CAP / 4; ++w) code[w] = sarg[w] = 0;
        len = 0;
        n_loads = 0;
    }
    __device__ __forceinline__ int code_at(int t) const {
        return (__builtin_amdgcn_readfirstlane(code[t >> 2]) >> ((t & 3) * 8)) & 0xff;
    }
    __device__ __forceinline__ int sarg_at(int t) const {
        return (__builtin_amdgcn_readfirstlane(sarg[t >> 2]) >> ((t & 3) * 8)) & 0xff;
    }
};
using InterpProg = InterpCodes<SALT_MAX_TOKENS>;
using InterpProg2 = InterpCodes<2 * SALT_MAX_TOKENS>;

// LDS bytes a workgroup of kBlock lanes needs for a program of stack depth
// `need` with EL values of `elem` bytes per lane.
inline size_t interp_lds_bytes(int need, int el, size_t elem) {
    return need > 1 ? (size_t)(need - 1) * el * elem * kBlock : 0;
}

// Run program `g` for EL elements per lane. get(k, j) yields element j of
// operand k (k < NL); `lds` is this workgroup's stack area. On return tos
// holds the value of the last slot written (the result, for one program).
template <int EL, int NL, class C, class Get, class Prog>
__device__ __forceinline__ void interp_run(const Prog &g, const C *sc, const Get &get, C (&tos)[EL], C *lds) {
    const int lane = threadIdx.x;
    for (int t = 0; t < g.len; ++t) {
        const int code = g.code_at(t);
        if (code < 72) {  // push: LOAD or SCALAR into slot s
            const int s = code & 7;
            if (s > 0) {
#pragma unroll
                for (int j = 0; j < EL; ++j) lds[((s - 1) * EL + j) * kBlock + lane] = tos[j];
            }
            if (code < 64) {
                switch (code >> 3) {
#define SALT_LOAD_K(k)                                                            \
    case k:                                                                       \
        if constexpr ((k) < NL) {                                                 \
            _Pragma("unroll") for (int j = 0; j < EL; ++j) tos[j] = get(k, j);    \
        }                                                                         \
        break;
                    SALT_LOAD_K(0) SALT_LOAD_K(1) SALT_LOAD_K(2) SALT_LOAD_K(3)
                    SALT_LOAD_K(4) SALT_LOAD_K(5) SALT_LOAD_K(6) SALT_LOAD_K(7)
#undef SALT_LOAD_K
                    default:
                        break;
                }
            } else {
                const C v = sc[g.sarg_at(t)];
#pragma unroll
                for (int j = 0; j < EL; ++j) tos[j] = v;
            }
        } else {  // binary: slot s (LDS) op slot s + 1 (top) -> slot s (top)
            const int op = (code - 72) >> 3, s = (code - 72) & 7;
            const C *left = lds + (size_t)s * EL * kBlock + lane;
            if (op == 0) {
#pragma unroll
                for (int j = 0; j < EL; ++j) tos[j] = left[j * kBlock] + tos[j];
            } else if (op == 1) {
#pragma unroll
                for (int j = 0; j < EL; ++j) tos[j] = left[j * kBlock] - tos[j];
            } else {
#pragma unroll
                for (int j = 0; j < EL; ++j) tos[j] = left[j * kBlock] * tos[j];
            }
        }
    }
}

// LDS one workgroup may take for the interpreter stack.
constexpr size_t kInterpLdsMax = 64 * 1024;

// Chunks per lane per program run: the largest power of two <= `want` whose
// stack fits in kInterpLdsMax (1 always fits: 7 rows x 8 values x 4 bytes x
// 256 lanes at most).
inline int interp_fit_unroll(int want, int need, int V, size_t elem) {
    int u = want >= 8 ? 8 : want >= 4 ? 4 : want >= 2 ? 2 : 1;
    while (u > 1 && interp_lds_bytes(need, u * V, elem) > kInterpLdsMax) u >>= 1;
    return u;
}

// Smallest of 2, 4, 8 that is >= v (v <= 8).
inline int interp_bound(int v) { return v <= 2 ? 2 : v <= 4 ? 4 : 8; }

}  // namespace salt
