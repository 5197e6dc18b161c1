// launch.hpp -- host-side interface between the C ABI and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "program.hpp"
#include "salt.h"

namespace salt {

// One element-wise launch: canonical operand pointers and scalars, shape and
// tuning knobs.
struct EvalLaunch {
    const void *ops[SALT_MAX_OPERANDS];
    double sc[SALT_MAX_SCALARS];
    void *out;
    int64_t n;
    int32_t vec;          // all arrays 16-byte aligned
    int32_t unroll;       // 16-byte chunks per operand per lane per tile
    int32_t nontemporal;  // streaming loads/stores
    int64_t blocks;       // 0 = one workgroup per tile, else grid size
    void *stream;
};

using EvalFn = hipError_t (*)(const EvalLaunch &);

// Grid of an element-wise launch whose tiles hold `tile` elements: one
// workgroup per whole tile (or L.blocks of them, grid-stride), else enough
// for the per-element loop (at most 8192 or L.blocks).
int64_t eval_grid(const EvalLaunch &L, int64_t tile);

// Ahead-of-time kernel launcher for catalogue tree `id` and `dtype`, or null.
EvalFn catalogue_launcher(int id, int dtype);
// Postfix form of catalogue tree `id` (canonical numbering) and its name;
// returns its length, or -1 for an unknown id.
int catalogue_program(int id, uint32_t *tokens, int cap, const char **name);
// Generic interpreter launch for a compiled program.
hipError_t launch_interp(const EvalLaunch &L, const Program &p, int dtype);

// Reductions (reduce.hip): what each element contributes.
enum ReduceMode { kModeDot = 0, kModeNrm2 = 1, kModeAsum = 2 };

struct ReduceLaunch {
    const void *x;
    const void *y;  // == x for nrm2 and asum
    void *result;
    double *ws;     // one binary64 partial per tile
    int64_t n;
    int32_t vec;
    int32_t unroll;     // chunks per lane per load burst
    int32_t nontemporal;
    int64_t blocks;     // 0 = one workgroup per tile, else grid size
    int32_t mode;       // ReduceMode
    int32_t passes;     // bit 0: pass 1 (partials into ws), bit 1: pass 2 (ws -> result)
    int64_t n_partials; // pass 2 alone: the partials in ws
    void *stream;
};
int64_t reduce_tile_elems(int dtype);
hipError_t launch_reduce(const ReduceLaunch &L, int dtype);

// dot / nrm2 of expressions (reduce.hip): operands in the caller's numbering.
struct ReduceExprLaunch {
    const void *ops[SALT_MAX_OPERANDS];
    double sc[SALT_MAX_SCALARS];
    void *result;
    double *ws;
    int64_t n;
    int32_t vec;
    uint32_t mask;
    int32_t unroll;  // chunks per lane per interpreter run: 2, 4, 8
    int32_t nontemporal;
    int64_t blocks;
    int32_t nrm2;
    void *stream;
};
hipError_t launch_reduce_expr(const ReduceExprLaunch &L, const Program &px, const Program *py, int dtype);
// Ahead-of-time reduction pair `id` (expr.hpp, SALT_RCATALOGUE): L.ops and
// L.sc in the pair's canonical numbering; L.mask is unused.
hipError_t launch_reduce_tree(const ReduceExprLaunch &L, int id, int dtype);
// The reduction pair that (P, Q) is, with operands and scalars renumbered
// (op_map[k] / sc_map[j]: the caller's index of canonical operand k /
// scalar j; *n_scalars, if not null, the distinct scalars read), or -1. Q
// is null for nrm2. A dot pair also matches with P and Q exchanged (the
// product is symmetric).
int route_pair(const uint32_t *px, int32_t lx, const uint32_t *py, int32_t ly, int32_t *op_map,
               int32_t *sc_map, int32_t *n_scalars);

// The plain read/write stream of salt_stream_reference (stream_ref.hip);
// *err receives the message of a failure.
salt_status stream_reference_impl(int32_t reads, int32_t writes, const void *const *inputs, void *output,
                                  int64_t bytes, void *stream, std::string *err);

}  // namespace salt
