// stream_ref.hip -- a plain streaming kernel used as a measured reference for
// the bandwidth one read/write mix reaches on the device (salt_stream_reference).
//
// It is deliberately the simplest possible stream: one 16-byte chunk per
// lane, one launch-wide pass, no loop, no expression machinery and no
// floating point (the R input chunks are combined by integer xor), with
// non-temporal loads and stores. Whatever it reaches for R reads and W
// writes per chunk is the ceiling that mix gives any kernel written this
// way; the fused-evaluation kernels are compared against it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "device.hpp"
#include "salt.h"

namespace salt {
namespace {

constexpr int kMaxRefReads = 6;

struct StreamRefArgs {
    const u32x4 *in[kMaxRefReads];
    u32x4 *out;
    int64_t chunks;
    int32_t never;  // always 0: keeps the loads of a read-only stream alive
};

template <int R, bool W>
__global__ __launch_bounds__(kBlock) void k_stream_ref(StreamRefArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.chunks) return;
    u32x4 v = ld16<true>(a.in[0] + i);
#pragma unroll
    for (int k = 1; k < R; ++k) v ^= ld16<true>(a.in[k] + i);
    if constexpr (W) st16<true>(a.out + i, v);
    else if (a.never && v[0] == 0u && v[1] == 0u) st16<true>(a.out + i, v);
}

template <int R>
hipError_t launch_ref(const StreamRefArgs &a, int writes, hipStream_t s) {
    const int64_t blocks = (a.chunks + kBlock - 1) / kBlock;
    if (writes)
        hipLaunchKernelGGL((k_stream_ref<R, true>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_stream_ref<R, false>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace

salt_status stream_reference_impl(int32_t reads, int32_t writes, const void *const *inputs, void *output,
                                  int64_t bytes, void *stream, std::string *err) {
    auto bad = [&](const char *m) {
        *err = m;
        return SALT_ERR_ARG;
    };
    if (reads < 1 || reads > kMaxRefReads) return bad("reads outside 1..6");
    if (writes < 0 || writes > 1) return bad("writes outside 0..1");
    if (bytes < 0 || bytes % 16) return bad("bytes must be a non-negative multiple of 16");
    if (bytes / 16 > (int64_t)kBlock * 0x7fffffffLL) return bad("too many bytes for one launch");
    if (bytes == 0) return SALT_OK;
    if (!inputs) return bad("inputs is NULL");
    StreamRefArgs a{};
    for (int k = 0; k < reads; ++k) {
        if (!inputs[k] || ((uintptr_t)inputs[k] & 15u)) return bad("an input is NULL or not 16-byte aligned");
        a.in[k] = (const u32x4 *)inputs[k];
    }
    if (writes && (!output || ((uintptr_t)output & 15u))) return bad("output is NULL or not 16-byte aligned");
    a.out = (u32x4 *)output;
    a.chunks = bytes / 16;
    a.never = 0;
    hipError_t e;
    hipStream_t s = (hipStream_t)stream;
    switch (reads) {
        case 1: e = launch_ref<1>(a, writes, s); break;
        case 2: e = launch_ref<2>(a, writes, s); break;
        case 3: e = launch_ref<3>(a, writes, s); break;
        case 4: e = launch_ref<4>(a, writes, s); break;
        case 5: e = launch_ref<5>(a, writes, s); break;
        default: e = launch_ref<6>(a, writes, s); break;
    }
    if (e != hipSuccess) {
        *err = std::string("HIP error: ") + hipGetErrorString(e);
        return SALT_ERR_DEVICE;
    }
    return SALT_OK;
}

}  // namespace salt
