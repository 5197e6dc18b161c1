// jit.hpp -- trees outside the catalogue compiled at run time (hipRTC).
//
// The paper builds every expression tree at compile time (Sec. 2); a tree
// that only arrives at run time would otherwise run on the interpreter. Here
// its canonical postfix form becomes a tree type of expr.hpp, and hipRTC
// instantiates the library's own element-wise kernel template for it
// (eval_tree.hpp, whose text and that of the headers it includes are
// embedded in the library at build time) for gfx950, with the library's
// build rules (contraction off, packed binary32 instructions off). The code
// is cached per (tree, element type), loaded per device on first use and
// launched instead of the interpreter. Same operations in the same order:
// the results are bit-identical to the interpreter's and the oracle's.
//
// Compiling takes about a second, so in the automatic mode a tree
// runs on the interpreter at its first call of at least kJitAutoMinElems
// elements and is compiled (on the calling thread) at its second, which then
// runs the compiled kernel, as do all later calls: a tree used once costs
// nothing, a tree used repeatedly pays one compile. The explicit mode
// compiles only what the caller asks for (salt_jit_compile).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "batch.hpp"
#include "launch.hpp"
#include "program.hpp"

namespace salt {

enum JitMode { kJitOff = 0, kJitExplicit = 1, kJitAuto = 2 };
constexpr int64_t kJitAutoMinElems = (int64_t)1 << 16;

// HIP source of the kernels for canonical program p (it includes the
// embedded headers and names the tree's type).
std::string jit_source(const Program &p, int dtype);

// A reduction pair in canonical numbering (operands and scalars numbered by
// first appearance in P, then in Q); Q is empty for nrm2(P).
struct PairTrees {
    uint32_t p[SALT_MAX_TOKENS], q[SALT_MAX_TOKENS];
    int lp = 0, lq = 0;
    bool nrm2 = false;
    int n_loads = 0;  // distinct operands read by P and Q
};

// HIP source of the pair's pass-1 kernels for element type dtype (it
// includes the embedded headers).
std::string jit_pair_source(const PairTrees &t, int dtype);

// Launch pass 1 of the pair's compiled kernel if it is compiled (same rules
// as jit_try_launch); *ran tells whether it did. L holds the pair's
// canonical operands and scalars, its workspace and result; when the
// reduction fits one tile, pass 1 stores the result itself, else the caller
// runs pass 2 over the partials.
hipError_t jit_try_reduce(const ReduceExprLaunch &L, const PairTrees &t, int dtype, bool *ran);
salt_status jit_compile_pair(const PairTrees &t, int dtype, std::string *err);
std::vector<char> jit_pair_code(const PairTrees &t, int dtype);
int jit_pair_ready(const PairTrees &t, int dtype);

// Batched launches (salt_batch_*) of a tree outside the catalogue: the
// library's batched kernel template (batch_device.hpp, embedded like the
// reduction headers) instantiated for the tree, with or without the fused
// dot (one module each), in every variant of chunks per burst and
// streaming hints; the per-item combine of the dots is the library's. A
// batched plan compiles its tree when it is created, so these do not
// depend on the mode.
std::string jit_batch_source(const Program &p, int dtype);
salt_status jit_compile_batch(const Program &p, int dtype, bool dot, std::string *err);
// Load the compiled tree's module on the current device (outside capture).
hipError_t jit_batch_load(const Program &p, int dtype, bool dot);
// Launch the batched kernel (and the combine when L.any_dot) of a compiled
// tree; loads its module on the current device first, which is refused
// (hipErrorStreamCaptureUnsupported) while L.stream is being captured.
hipError_t jit_batch_launch(const BatchLaunch &L, const Program &p, int dtype);
std::vector<char> jit_batch_code(const Program &p, int dtype, bool dot);

// Launch p's compiled kernel if it is compiled (loading it on the current
// device first unless the stream is being captured); *ran tells whether it
// did. In the automatic mode a tree's second large call compiles it first.
// L holds canonical operands and scalars, as for the catalogue kernels.
hipError_t jit_try_launch(const EvalLaunch &L, const Program &p, int dtype, bool *ran);

// Compile p for dtype now (blocking; no GPU needed). SALT_OK when the code
// object is in the cache, SALT_ERR_UNSUPPORTED with hipRTC's log otherwise.
salt_status jit_compile(const Program &p, int dtype, std::string *err);

// Copy of the compiled code object (empty if not compiled).
std::vector<char> jit_code(const Program &p, int dtype);

// 1: compiled (ready to load and launch), 0: not (yet) compiled.
int jit_ready(const Program &p, int dtype);

void jit_set_mode(int mode);
int jit_mode();

}  // namespace salt
