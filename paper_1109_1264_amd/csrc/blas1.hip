// blas1.hip -- the BLAS level-1 interface with increments (strided vectors)
// and iamax, for gfx950.
//
// The paper measures its fused kernels against BLAS level-1 routines (Sec. 1,
// the BLAS interface; Sec. 5, xDOT, xSCAL, xAXPY and xCOPY). BLAS vectors
// carry an increment: element i of an n-element vector with increment inc
// sits at x[i*inc] for inc >= 0 and at x[(n-1-i)*|inc|] for inc < 0. Unit
// increments go to the contiguous kernels (eval.hip, reduce_kernels.hpp);
// these kernels serve the other increments.
//
//  * k_strided_map: scal (x = alpha x), axpy (y = alpha x + y) and copy, one
//    element per lane per step, grid-stride. Each element is loaded, computed
//    and stored exactly as the contiguous kernels do (compute type, one
//    rounding per operation, one narrowing at the store), so the bits match.
//  * k_reduce_strided: pass 1 of dot / nrm2 / asum with the contiguous
//    kernel's canonical order (tile, lane, chunk, slot), element by element;
//    pass 2 is the contiguous one. A strided reduction therefore has the same
//    bits as the contiguous reduction of the gathered vectors.
//  * k_iamax_pass1 / k_iamax_pass2a / k_iamax_pass2: first index of the
//    largest magnitude.
//    The order "larger magnitude, then smaller index" is total, so the tree
//    of comparisons gives the scan's answer whatever its shape. A NaN never
//    wins (its key is below every magnitude) except as element 0, which the
//    scan keeps because nothing compares greater than it.
#include "blas1.hpp"
#include "reduce_kernels.hpp"

namespace salt {

__device__ __forceinline__ int64_t blas_off(int64_t i, int64_t n, int64_t inc) {
    return inc >= 0 ? i * inc : (n - 1 - i) * (-inc);
}

// ---------------------------------------------------------------------------
// element-wise: scal, axpy, copy
// ---------------------------------------------------------------------------

template <int DT, int OP>
__global__ __launch_bounds__(kBlock) void k_strided_map(StridedMapLaunch a) {
    using C = typename Tr<DT>::C;
    const C alpha = (C)a.alpha;  // rounded once to the compute type (RNE)
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += step) {
        const int64_t ox = blas_off(i, a.n, a.incx);
        if constexpr (OP == kMapScal) {
            Tr<DT>::st1(a.y, ox, alpha * Tr<DT>::ld1(a.x, ox));
        } else {
            const int64_t oy = blas_off(i, a.n, a.incy);
            const C p = alpha * Tr<DT>::ld1(a.x, ox);
            Tr<DT>::st1(a.y, oy, p + Tr<DT>::ld1(a.y, oy));
        }
    }
}

template <class S>
__global__ __launch_bounds__(kBlock) void k_strided_copy(StridedMapLaunch a) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += step)
        ((S *)a.y)[blas_off(i, a.n, a.incy)] = ((const S *)a.x)[blas_off(i, a.n, a.incx)];
}

static int64_t map_grid(int64_t n) {
    const int64_t g = (n + kBlock - 1) / kBlock;
    return g < 8192 ? g : 8192;  // 32 workgroups per CU, grid-stride beyond
}

template <int DT>
static hipError_t launch_map_dt(const StridedMapLaunch &L) {
    const dim3 grid((unsigned)map_grid(L.n)), block(kBlock);
    if (L.op == kMapScal)
        hipLaunchKernelGGL((k_strided_map<DT, kMapScal>), grid, block, 0, (hipStream_t)L.stream, L);
    else
        hipLaunchKernelGGL((k_strided_map<DT, kMapAxpy>), grid, block, 0, (hipStream_t)L.stream, L);
    return hipGetLastError();
}

hipError_t launch_strided_map(const StridedMapLaunch &L, int dtype) {
    if (L.n <= 0) return hipSuccess;
    if (L.op == kMapCopy) {
        const dim3 grid((unsigned)map_grid(L.n)), block(kBlock);
        switch (dtype) {
            case SALT_F64:
                hipLaunchKernelGGL((k_strided_copy<uint64_t>), grid, block, 0, (hipStream_t)L.stream, L);
                break;
            case SALT_F32:
                hipLaunchKernelGGL((k_strided_copy<uint32_t>), grid, block, 0, (hipStream_t)L.stream, L);
                break;
            default:
                hipLaunchKernelGGL((k_strided_copy<uint16_t>), grid, block, 0, (hipStream_t)L.stream, L);
                break;
        }
        return hipGetLastError();
    }
    switch (dtype) {
        case SALT_F64: return launch_map_dt<SALT_F64>(L);
        case SALT_F32: return launch_map_dt<SALT_F32>(L);
        case SALT_BF16: return launch_map_dt<SALT_BF16>(L);
        case SALT_F16: return launch_map_dt<SALT_F16>(L);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// strided dot / nrm2 / asum, pass 1
// ---------------------------------------------------------------------------

// Chunks loaded per burst: independent loads in flight before accumulating.
constexpr int kStridedBurst = 4;

template <int DT, int MODE>
__global__ __launch_bounds__(kBlock) void k_reduce_strided(StridedReduceLaunch a) {
    using C = typename Tr<DT>::C;
    constexpr int V = Tr<DT>::V;
    constexpr int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (a.n + T - 1) / T;
    __shared__ double lds[kBlock / 64];
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        Acc<DT> acc[V];
        const int64_t c0 = t * ((int64_t)kBlock * kChunksPerLane) + threadIdx.x;
#pragma unroll
        for (int it0 = 0; it0 < kChunksPerLane; it0 += kStridedBurst) {
            C xs[kStridedBurst][V], ys[kStridedBurst][V];
#pragma unroll
            for (int u = 0; u < kStridedBurst; ++u)
#pragma unroll
                for (int p = 0; p < V; ++p) {
                    const int64_t j = (c0 + (int64_t)(it0 + u) * kBlock) * V + p;
                    const bool in = j < a.n;
                    xs[u][p] = in ? Tr<DT>::ld1(a.x, blas_off(j, a.n, a.incx)) : (C)0;
                    if constexpr (MODE == kModeDot) ys[u][p] = in ? Tr<DT>::ld1(a.y, blas_off(j, a.n, a.incy)) : (C)0;
                    else ys[u][p] = xs[u][p];
                }
#pragma unroll
            for (int u = 0; u < kStridedBurst; ++u)
#pragma unroll
                for (int p = 0; p < V; ++p) acc_add<DT, MODE>(acc[p], xs[u][p], ys[u][p]);
        }
        const double v = block_sum<kBlock / 64>(lane_value<DT>(acc), lds);
        if (threadIdx.x == 0) a.ws[t] = v;
    }
}

template <int DT, int MODE>
static hipError_t launch_strided_reduce_m(const StridedReduceLaunch &L) {
    constexpr int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (L.n + T - 1) / T;
    if (n_tiles > 0) {
        const int64_t grid = n_tiles < 0x7fffffff ? n_tiles : 0x7fffffff;
        hipLaunchKernelGGL((k_reduce_strided<DT, MODE>), dim3((unsigned)grid), dim3(kBlock), 0,
                           (hipStream_t)L.stream, L);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_reduce_pass2<DT, MODE == kModeNrm2>), dim3(1), dim3(kFinalBlock), 0,
                       (hipStream_t)L.stream, (const double *)L.ws, n_tiles, L.result);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_strided_reduce_dt(const StridedReduceLaunch &L) {
    switch (L.mode) {
        case kModeNrm2: return launch_strided_reduce_m<DT, kModeNrm2>(L);
        case kModeAsum: return launch_strided_reduce_m<DT, kModeAsum>(L);
        default: return launch_strided_reduce_m<DT, kModeDot>(L);
    }
}

hipError_t launch_strided_reduce(const StridedReduceLaunch &L, int dtype) {
    switch (dtype) {
        case SALT_F64: return launch_strided_reduce_dt<SALT_F64>(L);
        case SALT_F32: return launch_strided_reduce_dt<SALT_F32>(L);
        case SALT_BF16: return launch_strided_reduce_dt<SALT_BF16>(L);
        case SALT_F16: return launch_strided_reduce_dt<SALT_F16>(L);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// iamax
// ---------------------------------------------------------------------------

template <int DT>
struct Amax {
    using K = typename Tr<DT>::C;  // magnitudes compare exactly in the compute type
    K key;
    int64_t idx;
    // A magnitude, or -1 for NaN (below every magnitude).
    __device__ __forceinline__ static K key_of(K v) { return v != v ? (K)-1 : (v < (K)0 ? -v : v); }
    __device__ __forceinline__ bool beats(const Amax &o) const {
        return key > o.key || (key == o.key && idx < o.idx);
    }
    __device__ __forceinline__ void take(K k, int64_t i) {
        const Amax c{k, i};
        if (c.beats(*this)) *this = c;
    }
    // Best of the wave, in every lane (xor butterfly; the order is total).
    __device__ __forceinline__ void wave_best() {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const Amax o{__shfl_xor(key, off, 64), __shfl_xor(idx, off, 64)};
            if (o.beats(*this)) *this = o;
        }
    }
};

// Best of a workgroup of W waves; every thread returns it. Ends with a
// barrier, so the LDS may be reused.
template <int DT, int W>
__device__ __forceinline__ Amax<DT> block_best(Amax<DT> b, typename Amax<DT>::K *lkey, int64_t *lidx) {
    b.wave_best();
    if ((threadIdx.x & 63) == 0) {
        lkey[threadIdx.x >> 6] = b.key;
        lidx[threadIdx.x >> 6] = b.idx;
    }
    __syncthreads();
    Amax<DT> r{lkey[0], lidx[0]};
#pragma unroll
    for (int w = 1; w < W; ++w) r.take(lkey[w], lidx[w]);
    __syncthreads();
    return r;
}

// Pass 1: per tile of T elements (the reductions' tile), the index of its
// best element. Each lane visits its elements in increasing index order, so a
// plain "greater magnitude" test keeps the first of equal magnitudes, and a
// NaN fails the test; the lane starts from its first element with key -1, so
// a lane of NaNs still names one of its own elements (which pass 2 rates
// below every magnitude). Unit stride with aligned data loads whole 16-byte
// chunks.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_iamax_pass1(IamaxLaunch a) {
    using K = typename Amax<DT>::K;
    constexpr int V = Tr<DT>::V;
    constexpr int64_t T = tile_elems<DT>();
    constexpr int B = 8;  // chunks per load burst
    const int64_t n_tiles = (a.n + T - 1) / T;
    __shared__ K lkey[kBlock / 64];
    __shared__ int64_t lidx[kBlock / 64];
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t c0 = t * ((int64_t)kBlock * kChunksPerLane) + threadIdx.x;
        const int64_t j0 = c0 * V;  // this lane's first element
        Amax<DT> best{j0 < a.n ? (K)-1 : (K)-2, j0 < a.n ? j0 : INT64_MAX};
        const bool whole = a.vec && (t + 1) * T <= a.n;
        if (whole) {
#pragma unroll
            for (int it0 = 0; it0 < kChunksPerLane; it0 += B) {
                u32x4 raw[B];
#pragma unroll
                for (int u = 0; u < B; ++u) raw[u] = ld16<true>((const u32x4 *)a.x + c0 + (int64_t)(it0 + u) * kBlock);
#pragma unroll
                for (int u = 0; u < B; ++u)
#pragma unroll
                    for (int p = 0; p < V; ++p) {
                        const K v = Tr<DT>::get(raw[u], p);
                        const K m = v < (K)0 ? -v : v;
                        if (m > best.key) {
                            best.key = m;
                            best.idx = (c0 + (int64_t)(it0 + u) * kBlock) * V + p;
                        }
                    }
            }
        } else {
            for (int it = 0; it < kChunksPerLane; ++it)
#pragma unroll
                for (int p = 0; p < V; ++p) {
                    const int64_t j = (c0 + (int64_t)it * kBlock) * V + p;
                    if (j < a.n) {
                        const K v = Tr<DT>::ld1(a.x, j * a.inc);
                        const K m = v < (K)0 ? -v : v;
                        if (m > best.key) {
                            best.key = m;
                            best.idx = j;
                        }
                    }
                }
        }
        best = block_best<DT, kBlock / 64>(best, lkey, lidx);
        if (threadIdx.x == 0) a.ws[t] = best.idx;
    }
}

// Pass 2a (many tiles): workgroup b rates candidates b*1024 ... b*1024+1023,
// one gather per lane, and writes its winner over the first of them (a slot
// no other workgroup reads). A single workgroup doing every gather would be
// limited by one CU's rate of cache-line requests.
template <int DT>
__global__ __launch_bounds__(kFinalBlock) void k_iamax_pass2a(IamaxLaunch a, int64_t count) {
    using K = typename Amax<DT>::K;
    __shared__ K lkey[kFinalBlock / 64];
    __shared__ int64_t lidx[kFinalBlock / 64];
    const int64_t t = (int64_t)blockIdx.x * kFinalBlock + threadIdx.x;
    Amax<DT> best{(K)-2, INT64_MAX};
    if (t < count) {
        const int64_t j = a.ws[t];
        best = Amax<DT>{Amax<DT>::key_of(Tr<DT>::ld1(a.x, j * a.inc)), j};
    }
    best = block_best<DT, kFinalBlock / 64>(best, lkey, lidx);
    if (threadIdx.x == 0) a.ws[(int64_t)blockIdx.x * kFinalBlock] = best.idx;
}

// Pass 2: one workgroup over the candidates ws[0], ws[stride], ... (count of
// them); writes the index, 0 when element 0 is NaN, -1 for an empty vector.
template <int DT>
__global__ __launch_bounds__(kFinalBlock) void k_iamax_pass2(IamaxLaunch a, int64_t count, int64_t stride) {
    using K = typename Amax<DT>::K;
    __shared__ K lkey[kFinalBlock / 64];
    __shared__ int64_t lidx[kFinalBlock / 64];
    if (a.n < 1) {
        if (threadIdx.x == 0) *a.result = -1;
        return;
    }
    const K x0 = Tr<DT>::ld1(a.x, 0);
    if (x0 != x0) {
        if (threadIdx.x == 0) *a.result = 0;
        return;
    }
    Amax<DT> best{(K)-2, INT64_MAX};
    // Candidates eight at a time: their indices, then their values, each as
    // one round of independent loads.
    constexpr int Q = 8;
    for (int64_t c0 = threadIdx.x; c0 < count; c0 += Q * kFinalBlock) {
        int64_t j[Q];
        K v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t c = c0 + (int64_t)q * kFinalBlock;
            j[q] = c < count ? a.ws[c * stride] : -1;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = j[q] >= 0 ? Tr<DT>::ld1(a.x, j[q] * a.inc) : (K)0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (j[q] >= 0) best.take(Amax<DT>::key_of(v[q]), j[q]);
    }
    best = block_best<DT, kFinalBlock / 64>(best, lkey, lidx);
    if (threadIdx.x == 0) *a.result = best.idx;
}

template <int DT>
static hipError_t launch_iamax_dt(const IamaxLaunch &L) {
    constexpr int64_t T = tile_elems<DT>();
    const int64_t n_tiles = L.n > 0 ? (L.n + T - 1) / T : 0;
    int64_t count = n_tiles, stride = 1;
    if (n_tiles > 0) {
        const int64_t grid = n_tiles < 0x7fffffff ? n_tiles : 0x7fffffff;
        hipLaunchKernelGGL((k_iamax_pass1<DT>), dim3((unsigned)grid), dim3(kBlock), 0, (hipStream_t)L.stream, L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (n_tiles > kFinalBlock) {
            count = (n_tiles + kFinalBlock - 1) / kFinalBlock;
            stride = kFinalBlock;
            hipLaunchKernelGGL((k_iamax_pass2a<DT>), dim3((unsigned)count), dim3(kFinalBlock), 0,
                               (hipStream_t)L.stream, L, n_tiles);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL((k_iamax_pass2<DT>), dim3(1), dim3(kFinalBlock), 0, (hipStream_t)L.stream, L, count, stride);
    return hipGetLastError();
}

hipError_t launch_iamax(const IamaxLaunch &L, int dtype) {
    switch (dtype) {
        case SALT_F64: return launch_iamax_dt<SALT_F64>(L);
        case SALT_F32: return launch_iamax_dt<SALT_F32>(L);
        case SALT_BF16: return launch_iamax_dt<SALT_BF16>(L);
        case SALT_F16: return launch_iamax_dt<SALT_F16>(L);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace salt
