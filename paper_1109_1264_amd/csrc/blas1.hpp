// blas1.hpp -- host-side interface of the strided BLAS level-1 kernels
// (blas1.hip). Element i of an n-element vector with increment inc is
// x[i*inc] for inc >= 0 and x[(n-1-i)*|inc|] for inc < 0; the host has
// checked every pointer, increment and span before a launch.
#pragma once

#include "launch.hpp"

namespace salt {

enum MapOp { kMapScal = 0, kMapAxpy = 1, kMapCopy = 2 };

// scal: y == x, x_i <- alpha x_i; axpy: y_i <- alpha x_i + y_i; copy: y_i <- x_i.
struct StridedMapLaunch {
    const void *x;
    int64_t incx;
    void *y;
    int64_t incy;
    int64_t n;
    double alpha;
    int32_t op;  // MapOp
    void *stream;
};
hipError_t launch_strided_map(const StridedMapLaunch &L, int dtype);

// dot / nrm2 / asum of strided vectors: pass 1 into ws (one binary64 per
// tile, the contiguous tiling), pass 2 into result.
struct StridedReduceLaunch {
    const void *x;
    int64_t incx;
    const void *y;  // dot only
    int64_t incy;
    void *result;
    double *ws;
    int64_t n;
    int32_t mode;  // ReduceMode
    void *stream;
};
hipError_t launch_strided_reduce(const StridedReduceLaunch &L, int dtype);

// iamax (inc >= 1): one candidate index per tile in ws, then the answer (an
// int64 in device memory).
struct IamaxLaunch {
    const void *x;
    int64_t inc;
    int64_t *result;
    int64_t *ws;
    int64_t n;
    int32_t vec;  // inc == 1 and x 16-byte aligned: whole tiles load 16-byte chunks
    void *stream;
};
hipError_t launch_iamax(const IamaxLaunch &L, int dtype);

}  // namespace salt
