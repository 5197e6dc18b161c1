/*
 * salt.h -- C ABI of libsalt: fused element-wise vector expressions, axpy,
 * dot and nrm2 on one AMD Instinct MI355X (gfx950).
 *
 * Method: Progsch, Ineichen and Adelmann, "A New Vectorization Technique for
 * Expression Templates in C++" (SALT). An expression over vectors is kept as
 * a tree and evaluated lazily, in one loop over the elements, when it is
 * assigned or reduced by a dot product or a norm (Sec. 2, Fig. 1); the loop
 * issues a burst of loads, then the operations, then the stores (Sec. 4.3).
 * Here the tree travels as a postfix program and the loop is a GPU kernel.
 *
 * Conventions shared by every entry point:
 *  - Data pointers (operands, outputs, workspaces, results) are DEVICE
 *    pointers owned by the caller; the library keeps none of them after the
 *    call returns and allocates no device memory on these paths.
 *  - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the default
 *    stream) and the call returns without waiting. Outputs, including the
 *    device scalar written by dot and nrm2, are valid once the stream has
 *    reached that point.
 *  - Vectors are contiguous, unit stride, one element type per call.
 *    Lengths are int64; n == 0 is a no-op for eval/axpy and yields 0 for
 *    dot/nrm2; n < 0 is SALT_ERR_ARG.
 *  - Every argument or program error is reported before anything is
 *    enqueued, with no partial effect. A failed launch returns
 *    SALT_ERR_DEVICE. No C++ exception crosses this interface.
 *    salt_last_error() gives a thread-local message for the last failure.
 *  - Calls may come from several host threads at once: the library's own
 *    state (the tuning table, the cache of run-time compiled kernels) is
 *    guarded, and calls on different streams may run concurrently on the
 *    device. A caller's buffers are its own to order: two calls that write
 *    the same output or workspace on unordered streams race (as do
 *    overlapping salt_dot_noalloc calls, which share the library's buffer).
 *  - Any element alignment is accepted; 16-byte aligned arrays take the
 *    vectorised (16 B per lane) path, others a per-element path with the
 *    same results (the paper's non-specialised fallback loop, Sec. 4.2).
 */
#ifndef SALT_H
#define SALT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element (storage) types. F64 computes in binary64; F32, BF16 and F16
 * compute in binary32 (16-bit values are widened exactly on load and rounded
 * to nearest-even once on store). */
typedef enum { SALT_F64 = 0, SALT_F32 = 1, SALT_BF16 = 2, SALT_F16 = 3 } salt_dtype;

typedef enum {
    SALT_OK = 0,
    SALT_ERR_ARG = 1,         /* null pointer, bad length, bad dtype, overlap */
    SALT_ERR_PROGRAM = 2,     /* malformed postfix program                     */
    SALT_ERR_UNSUPPORTED = 3, /* valid request outside the library's limits    */
    SALT_ERR_WORKSPACE = 4,   /* workspace missing, misaligned or too small    */
    SALT_ERR_DEVICE = 5       /* HIP reported an error                         */
} salt_status;

/* Postfix program tokens: uint32 token = (arg << 8) | opcode.
 * LOAD k    pushes operands[k][i]
 * SCALAR j  pushes scalars[j], rounded once (nearest-even) to the compute type
 * ADD/SUB/MUL pop r, pop l, push (l op r), rounded once, never contracted
 *            into a fused multiply-add.
 * A program is valid when every token is one of these, binary tokens have
 * arg 0, k < n_operands, j < n_scalars, the stack never underflows, never
 * holds more than SALT_MAX_STACK values, and ends with exactly one value.
 * "Scale" is SCALAR j, <subtree>, MUL. */
enum {
    SALT_OP_LOAD = 1,
    SALT_OP_SCALAR = 2,
    SALT_OP_ADD = 3,
    SALT_OP_SUB = 4,
    SALT_OP_MUL = 5
};
#define SALT_TOKEN(op, arg) ((uint32_t)(((uint32_t)(arg) << 8) | (uint32_t)(op)))

#define SALT_MAX_TOKENS 64
#define SALT_MAX_OPERANDS 8
#define SALT_MAX_SCALARS 8
#define SALT_MAX_STACK 8

/* Fused element-wise evaluation (Sec. 2, Fig. 1; loop structure Sec. 4.3):
 *   out[i] = P(operands[0][i], ..., operands[n_operands-1][i]; scalars)
 * for 0 <= i < n, in one pass over memory: inputs read once, out written
 * once, intermediates kept in registers.
 *  prog        host array of prog_len tokens (1..SALT_MAX_TOKENS)
 *  operands    host array of n_operands device pointers (0..SALT_MAX_OPERANDS),
 *              each to n elements of `dtype`
 *  scalars     host array of n_scalars doubles (0..SALT_MAX_SCALARS)
 *  out         device pointer to n elements of `dtype`; may be identical to an
 *              operand pointer (in-place update) but must not partially
 *              overlap any operand (SALT_ERR_ARG).
 * Results are bit-identical to evaluating the postfix program element by
 * element in the compute type, in program order. */
salt_status salt_eval(const uint32_t *prog, int32_t prog_len,
                      const void *const *operands, int32_t n_operands,
                      const double *scalars, int32_t n_scalars,
                      void *out, int64_t n, salt_dtype dtype, void *hip_stream);

/* y <- alpha*x + y (Sec. 5, xAXPY): each element fl(fl(alpha*x) + y), alpha
 * rounded once to the compute type, no fused multiply-add. x and y are
 * device pointers to n elements; y is updated in place. */
salt_status salt_axpy(int64_t n, double alpha, const void *x, void *y,
                      salt_dtype dtype, void *hip_stream);

/* Bytes of device workspace that salt_dot / salt_nrm2 need for length n
 * (one binary64 partial per fixed-size tile of the input). 0 for n <= 0. */
size_t salt_reduce_workspace_bytes(int64_t n, salt_dtype dtype);

/* Dot product sum_i x[i]*y[i] (Sec. 2, reduction at the root of a tree;
 * Sec. 4.2, the reduction step). The summation order depends only on n and
 * dtype (fixed tiles, fixed in-tile order, fixed tree over tiles), so the
 * result is bit-reproducible across calls, launch shapes and batching.
 * Accumulation: binary64 for F64; for F32/BF16/F16 compensated binary32
 * (error-free products and sums) per lane, binary64 across lanes and tiles.
 *  result     device pointer to one double (F64) or one float (others)
 *  workspace  device buffer, 8-byte aligned, >= salt_reduce_workspace_bytes */
salt_status salt_dot(int64_t n, const void *x, const void *y, void *result,
                     void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream);

/* salt_dot without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc. Same arguments (minus the workspace), same
 * summation order and accumulation, and so the same result bits as
 * salt_dot. The tile partials go to a buffer inside the library: a
 * SALT_NOALLOC_MAX_PARTIALS-double (1 MiB) array on each GPU the library
 * runs on, held until the process ends. The call allocates nothing.
 *  - n may need at most SALT_NOALLOC_MAX_PARTIALS tiles, i.e.
 *    salt_reduce_workspace_bytes(n, dtype) <= 1 MiB: n <= 2^30 (F64),
 *    2^31 (F32), 2^32 (BF16/F16); beyond that SALT_ERR_UNSUPPORTED, before
 *    anything is enqueued.
 *  - Every call on one GPU shares that GPU's buffer, which keeps the last
 *    call's partials (pass 1 overwrites every partial that pass 2 reads, so
 *    nothing needs clearing). Calls that may overlap in time on one GPU
 *    (different streams with no ordering between them, or threads) race and
 *    give wrong results; calls ordered on one stream are safe.
 *  - The first call on a GPU looks up that GPU's buffer address with that
 *    GPU current (hipGetSymbolAddress); a failure there is SALT_ERR_DEVICE. */
#define SALT_NOALLOC_MAX_PARTIALS 131072
salt_status salt_dot_noalloc(int64_t n, const void *x, const void *y, void *result,
                             salt_dtype dtype, void *hip_stream);

/* Euclidean norm sqrt(sum_i x[i]^2), unscaled (the paper's "norm", Sec. 2),
 * with the same summation order, accumulation and arguments as salt_dot. */
salt_status salt_nrm2(int64_t n, const void *x, void *result,
                      void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream);

/* Lazy evaluation inside a reduction (Sec. 2: trees are evaluated where they
 * are needed, e.g. in a dot product or a norm): dot(P, Q) = sum_i P_i * Q_i
 * for two postfix programs P and Q over one operand list, and
 * nrm2(P) = sqrt(sum_i P_i^2), in one pass that reads each operand used by
 * either program once and writes no vector. The elements P_i and Q_i are the
 * values salt_eval would produce, and they are summed in salt_dot's order, so
 * the result has the same bits as salt_dot applied to the vectors salt_eval
 * would write (the product of two values is symmetric, so the order of P
 * and Q does not matter). Programs, operands and scalars are validated as
 * for salt_eval (operands need not all be used); workspace and result as for
 * salt_dot. One of P and Q must fit in SALT_MAX_STACK - 1 stack slots (it
 * runs on top of the other's result), else SALT_ERR_UNSUPPORTED. */
salt_status salt_dot_expr(const uint32_t *prog_x, int32_t len_x,
                          const uint32_t *prog_y, int32_t len_y,
                          const void *const *operands, int32_t n_operands,
                          const double *scalars, int32_t n_scalars, int64_t n,
                          void *result, void *workspace, size_t ws_bytes,
                          salt_dtype dtype, void *hip_stream);
salt_status salt_nrm2_expr(const uint32_t *prog, int32_t prog_len,
                           const void *const *operands, int32_t n_operands,
                           const double *scalars, int32_t n_scalars, int64_t n,
                           void *result, void *workspace, size_t ws_bytes,
                           salt_dtype dtype, void *hip_stream);

/* ---- BLAS level-1 with increments ------------------------------------------
 * The BLAS interface the paper measures against (Sec. 1; Sec. 5, xDOT,
 * xSCAL, xAXPY, xCOPY). A vector argument is (pointer, n, inc): element i
 * sits at x[i*inc] for inc >= 0 and at x[(n-1-i)*|inc|] for inc < 0, so the
 * pointer is always the lowest address and the vector spans
 * 1 + (n-1)*|inc| elements; inc = 0 repeats x[0] (inputs only). All
 * pointers are device pointers. Unit increments run the contiguous kernels
 * above (same bits); other increments run element-strided kernels with the
 * same arithmetic, so a strided call gives the bits the contiguous call
 * gives on the gathered vectors. The routines of one vector (scal, nrm2,
 * asum, iamax) treat inc <= 0 as the reference BLAS does: nothing is done,
 * or the result is 0 (nrm2, asum) or -1 (iamax). Errors (SALT_ERR_ARG): n < 0,
 * a NULL pointer with n > 0, a span past 2^59 elements, an output increment
 * of 0 with n > 1 (every element would land on one address). An output must
 * not overlap an input except as the very same vector (same pointer and
 * increment); this is not checked. Reductions take the workspace of
 * salt_reduce_workspace_bytes(n, dtype) and write the result type of
 * salt_dot. */

/* x_i <- alpha*x_i, alpha rounded once to the compute type. */
salt_status salt_scal(int64_t n, double alpha, void *x, int64_t incx,
                      salt_dtype dtype, void *hip_stream);

/* y_i <- x_i (bit copy). */
salt_status salt_copy(int64_t n, const void *x, int64_t incx, void *y, int64_t incy,
                      salt_dtype dtype, void *hip_stream);

/* y_i <- fl(fl(alpha*x_i) + y_i), as salt_axpy. */
salt_status salt_axpy_strided(int64_t n, double alpha, const void *x, int64_t incx,
                              void *y, int64_t incy, salt_dtype dtype, void *hip_stream);

/* sum_i x_i*y_i, sqrt(sum_i x_i^2) and sum_i |x_i|, with salt_dot's
 * summation order over the element index i and its accumulators. */
salt_status salt_dot_strided(int64_t n, const void *x, int64_t incx, const void *y, int64_t incy,
                             void *result, void *workspace, size_t ws_bytes,
                             salt_dtype dtype, void *hip_stream);
salt_status salt_nrm2_strided(int64_t n, const void *x, int64_t incx, void *result,
                              void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream);
salt_status salt_asum(int64_t n, const void *x, int64_t incx, void *result,
                      void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream);

/* Index (from 0) of the first element of largest magnitude, written to
 * *result (device int64). As in the reference BLAS scan, a NaN is never
 * chosen unless it is element 0 (then the answer is 0); -1 for n < 1 or
 * incx <= 0. The answer is unique, so it does not depend on the launch. */
salt_status salt_iamax(int64_t n, const void *x, int64_t incx, int64_t *result,
                       void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream);

/* ---- sharded reductions ------------------------------------------------------
 * The two passes of salt_dot / salt_nrm2 / salt_asum as separate calls, for a
 * vector split into shards (on several devices, or processed piecewise). A
 * shard boundary must fall on a tile boundary: every shard except the last
 * holds a multiple of salt_reduce_tile_elems(dtype) elements. Then the
 * shards' partials, placed side by side in shard order, are exactly the
 * partials of the whole vector, and combining them gives the bits of the
 * one-call result, for any number of shards (on several GPUs the partials,
 * 8 bytes per tile, are gathered to one device and combined there).
 *  mode  0: dot (x, y), 1: nrm2 (x), 2: asum (x); y is ignored unless dot. */

/* Pass 1 over the n elements of one shard: ceil(n / tile) binary64 partials,
 * in tile order, to `partials` (device, 8-byte aligned, not overlapping x or
 * y). Unit increments only. */
salt_status salt_reduce_partials(int32_t mode, int64_t n, const void *x, const void *y, double *partials,
                                 salt_dtype dtype, void *hip_stream);

/* Pass 2: the fixed combine of `count` partials (device) into the device
 * scalar `result` (double for F64, float otherwise; the square root for
 * nrm2). count = 0 gives 0. */
salt_status salt_reduce_combine(int32_t mode, const double *partials, int64_t count, void *result,
                                salt_dtype dtype, void *hip_stream);

/* ---- launch control (autotuning and introspection) ------------------------
 * The paper picks the number of instruction packages per loop by trial
 * (Sec. 4.3); here the equivalent knobs are chosen per tree, element type
 * and size by a measured tuning table, and can be forced for measurement.
 * None of them changes any result bit. */
typedef struct {
    int32_t unroll;      /* 16-byte chunks per operand per lane per burst:
                          * eval 1, 2, 4, 8; dot/nrm2 2, 4, 8, 16; batched
                          * 2, 4, 8; 0 = tuned */
    int32_t nontemporal; /* 1 streaming loads/stores, 0 normal, -1 = tuned */
    int64_t blocks;      /* workgroups: 0 = one per tile, >0 = grid-stride
                          * grid of that size, -1 = tuned */
} salt_launch_config;

/* salt_eval with explicit launch knobs (cfg NULL = tuned). */
salt_status salt_eval_ex(const uint32_t *prog, int32_t prog_len,
                         const void *const *operands, int32_t n_operands,
                         const double *scalars, int32_t n_scalars,
                         void *out, int64_t n, salt_dtype dtype, void *hip_stream,
                         const salt_launch_config *cfg);

/* salt_dot_expr / salt_nrm2_expr with explicit launch knobs (cfg NULL =
 * tuned; unroll 2, 4 or 8 chunks per interpreter run, 16 runs as 8). */
salt_status salt_dot_expr_ex(const uint32_t *prog_x, int32_t len_x,
                             const uint32_t *prog_y, int32_t len_y,
                             const void *const *operands, int32_t n_operands,
                             const double *scalars, int32_t n_scalars, int64_t n,
                             void *result, void *workspace, size_t ws_bytes,
                             salt_dtype dtype, void *hip_stream, const salt_launch_config *cfg);
salt_status salt_nrm2_expr_ex(const uint32_t *prog, int32_t prog_len,
                              const void *const *operands, int32_t n_operands,
                              const double *scalars, int32_t n_scalars, int64_t n,
                              void *result, void *workspace, size_t ws_bytes,
                              salt_dtype dtype, void *hip_stream, const salt_launch_config *cfg);

/* salt_dot / salt_nrm2 with explicit launch knobs (cfg NULL = tuned). */
salt_status salt_dot_ex(int64_t n, const void *x, const void *y, void *result,
                        void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream,
                        const salt_launch_config *cfg);
salt_status salt_nrm2_ex(int64_t n, const void *x, void *result,
                         void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream,
                         const salt_launch_config *cfg);

/* Elements per reduction tile for dtype (the unit of the fixed order). */
int64_t salt_reduce_tile_elems(salt_dtype dtype);

/* Load a tuning table (text; one "kind route dtype log2n unroll nontemporal
 * blocks" row per line, "#" comments; kind is eval, dot, nrm2 or batch; route is a
 * catalogue index or -1 for the interpreter). NULL reloads the default file
 * (SALT_TUNE_FILE, else salt_tuning.txt beside the library). Rows replace the
 * current table. Returns SALT_ERR_ARG if the file cannot be read or parsed. */
salt_status salt_tuning_load(const char *path);

/* The knobs a call would use (kind 0 eval, 1 dot, 2 nrm2, 3 batch; for a
 * batch, n is the total number of elements). */
salt_status salt_tuning_lookup(int32_t kind, int32_t route, salt_dtype dtype, int64_t n,
                               salt_launch_config *out);

/* Trees compiled ahead of time. salt_catalogue_program copies tree i's
 * canonical postfix form into tokens (up to cap) and returns its length, or
 * -1 for a bad index; *name (if non-NULL) receives its name. */
int32_t salt_catalogue_count(void);
int32_t salt_catalogue_program(int32_t i, uint32_t *tokens, int32_t cap, const char **name);

/* Which kernel a valid program runs on: *route = catalogue index, or -1 for
 * the generic interpreter. Host only. */
salt_status salt_program_route(const uint32_t *prog, int32_t prog_len,
                               int32_t n_operands, int32_t n_scalars, int32_t *route);

/* ---- batched evaluation --------------------------------------------------
 * Many independent evaluations of one tree, of uneven lengths, in one
 * persistent launch: every item is cut into the reduction's fixed tiles and
 * a grid of workgroups walks the flat list of all items' tiles. An item can
 * also ask for dot(operands[0], operands[1]), computed from the same loaded
 * registers (the operands are read once for both); its summation order is
 * that of salt_dot, so the result has the same bits as salt_dot alone. */
typedef struct {
    int64_t n;                                /* elements (>= 0)                     */
    const void *operands[SALT_MAX_OPERANDS];  /* device pointers, as for salt_eval   */
    double scalars[SALT_MAX_SCALARS];
    void *out;      /* device pointer to n elements, or NULL for no element-wise output */
    void *dot_out;  /* device scalar (double for F64, float otherwise) for
                     * dot(operands[0], operands[1]), or NULL */
} salt_batch_item;

typedef struct salt_batch_plan_s *salt_batch_plan;
typedef struct salt_graph_s *salt_graph;

/* Validate `count` items against one program and element type and build the
 * host side of the descriptor table. A catalogue tree (salt_catalogue_*)
 * runs its ahead-of-time batched kernels; any other tree has the same
 * kernel template compiled for it here, at plan creation (blocking, a few
 * seconds the first time per tree and type; cached for the process, same
 * bits), unless run-time compilation is off (salt_jit_set_mode), which
 * gives SALT_ERR_UNSUPPORTED, as does a failed compilation (log in
 * salt_last_error). An item with dot_out needs a program whose first two
 * operands read (in postfix order) are operands[0] and operands[1]. Every
 * check of salt_eval applies to every item. Items must not write to memory
 * another item reads or writes. On success *plan owns host memory only;
 * free it with salt_batch_plan_destroy. */
salt_status salt_batch_plan_create(const uint32_t *prog, int32_t prog_len,
                                   int32_t n_operands, int32_t n_scalars,
                                   const salt_batch_item *items, int32_t count,
                                   salt_dtype dtype, salt_batch_plan *plan);

/* Device bytes the plan needs: the descriptor table (uploaded once) and the
 * workspace (one binary64 per tile when any item has a dot, else 0), and the
 * number of tiles. */
salt_status salt_batch_plan_info(salt_batch_plan plan, size_t *table_bytes,
                                 size_t *ws_bytes, int64_t *tiles);

/* Copy the descriptor table into `table` (device, 256-byte aligned, at least
 * table_bytes) on `hip_stream` and wait for the copy. The plan keeps the
 * pointer: later launches read the table there. */
salt_status salt_batch_upload(salt_batch_plan plan, void *table, size_t table_bytes,
                              void *hip_stream);

/* Enqueue the batched kernel (and, when any item has a dot, the per-item
 * combine) on `hip_stream`. `workspace`: device, 8-byte aligned, >= ws_bytes
 * (may be NULL when ws_bytes is 0). cfg NULL = tuned. A plan of a tree
 * compiled at run time loads its kernels on the current device at its first
 * launch there; while `hip_stream` is being captured that load is refused
 * (SALT_ERR_DEVICE): launch it once first, or use salt_batch_graph_create,
 * which loads before it captures. */
salt_status salt_batch_launch(salt_batch_plan plan, void *workspace, size_t ws_bytes,
                              void *hip_stream, const salt_launch_config *cfg);

/* Capture salt_batch_launch into a HIP graph (on a private stream) and
 * instantiate it; salt_graph_launch replays it on any stream. The graph
 * holds the table, workspace and item pointers as they are now. */
salt_status salt_batch_graph_create(salt_batch_plan plan, void *workspace, size_t ws_bytes,
                                    const salt_launch_config *cfg, salt_graph *graph);
salt_status salt_graph_launch(salt_graph graph, void *hip_stream);
void salt_graph_destroy(salt_graph graph);
void salt_batch_plan_destroy(salt_batch_plan plan);

/* ---- serving ---------------------------------------------------------------
 * A request loop over expression evaluations whose operands stay resident
 * in device memory. Requests arrive over time (open loop, from a trace);
 * each is admitted when a slot is free and its output fits in the output
 * arena (first-fit; memory-based admission, FIFO order); admitted requests
 * are gathered into batched launches (per element type in the batch, one
 * launch with items of every tree mixed, or one launch per tree) on one of
 * several streams as soon as a stream can take more work,
 * so requests that arrive while others run are admitted and overlap with
 * them on the device (continuous batching). Completion times are the GPU
 * events of the batch, mapped to the host clock. Everything runs on the
 * calling thread; the call first waits for the device to be idle (work the
 * caller queued on any stream, such as filling the operands, completes
 * first) and returns when every request has completed or been rejected. */
typedef struct {
    void *arena;             /* device memory for outputs (caller-owned)      */
    size_t arena_bytes;
    void *table_arena;       /* device memory for descriptor tables           */
    size_t table_bytes;
    int32_t max_inflight;    /* requests admitted but not yet complete (slots) */
    int32_t n_streams;       /* 1..8 streams, default priority                */
    int32_t max_batch;       /* requests per batched launch                    */
    int32_t depth;           /* batches in flight per stream (1..4)           */
    int32_t release_on_complete; /* 1: free an output as soon as it completes;
                                  * 0: keep every output (results[i].out)    */
    int32_t grouping;        /* launches of one batch, per element type:
                              * 0 one mixed-tree launch; 1 one single-tree
                              * launch per tree; 2 one per tree when the
                              * type's requests in the batch hold at least
                              * SALT_SERVE_SPLIT_ELEMS elements, else mixed */
    const salt_launch_config *launch; /* knobs of every batched launch, as
                              * for salt_eval_ex (unroll 0, nontemporal -1,
                              * blocks -1: tuned), or NULL: all tuned, per
                              * launch by its tree, type and size; unroll
                              * 2, 4 or 8 (a mixed-tree launch runs 8 as 4) */
    int64_t range_bytes;     /* a group whose tiles hold more than twice this
                              * many bytes per operand runs as several
                              * launches over consecutive ranges of its tile
                              * list, each with the knobs of its size (same
                              * results); 0: 256 MiB, negative: never split */
} salt_server_config;
#define SALT_SERVE_SPLIT_ELEMS ((int64_t)1 << 26)

typedef struct {
    double arrival_s;                       /* seconds from the start of the run */
    int32_t tree;                           /* catalogue index                   */
    int32_t dtype;
    int64_t n;
    const void *operands[SALT_MAX_OPERANDS];  /* device pointers, as salt_eval   */
    double scalars[SALT_MAX_SCALARS];
} salt_request;

typedef struct {
    double arrival_s, admit_s, launch_s, complete_s;  /* seconds from the start */
    void *out;            /* the output in the arena (valid only when kept)     */
    int32_t status;       /* SALT_OK, or why the request was rejected          */
    int32_t batch;        /* index of the batched launch that ran it           */
} salt_request_result;

/* Run `count` requests (sorted by arrival_s) through the server and fill
 * results[0..count). Host memory for staging is allocated and freed inside
 * the call (pinned); no device memory is allocated. Returns SALT_ERR_ARG on a
 * bad configuration, SALT_ERR_DEVICE on a HIP failure; a bad request is
 * rejected with its own status and does not stop the others. */
salt_status salt_serve_trace(const salt_server_config *cfg, const salt_request *requests,
                             int32_t count, salt_request_result *results);

/* ---- trees outside the catalogue: run-time compilation --------------------
 * salt_eval runs a catalogue tree on its ahead-of-time kernel. Any other
 * tree runs on a kernel compiled for it at run time (hipRTC, gfx950, with
 * the library's own build rules: no contraction, no packed binary32
 * instructions) once that kernel is ready, and on the interpreter until
 * then; both give the same bits. Compiled kernels are cached per (tree in
 * canonical numbering, element type) for the life of the process and
 * loaded on a device at their first launch there (the runtime allocates
 * their code memory then; a launch on a stream being captured into a graph
 * does not load one and runs interpreted instead).
 * Modes: SALT_JIT_OFF (always the interpreter); SALT_JIT_EXPLICIT (only
 * trees passed to salt_jit_compile); SALT_JIT_AUTO (the default: a tree
 * runs interpreted at its first call of at least 65536 elements, and its
 * second such call compiles it on the calling thread, a one-time delay of
 * the order of a second, then runs it compiled, as do later calls). */
enum { SALT_JIT_OFF = 0, SALT_JIT_EXPLICIT = 1, SALT_JIT_AUTO = 2 };
#define SALT_ROUTE_COMPILED (-3)
salt_status salt_jit_set_mode(int32_t mode);

/* Compile the tree of `prog` for `dtype` now and cache it (blocking; needs
 * no GPU). SALT_OK also for a catalogue tree (nothing to do);
 * SALT_ERR_UNSUPPORTED with the compiler's log in salt_last_error() if
 * compilation fails. The program is validated as for salt_eval. */
salt_status salt_jit_compile(const uint32_t *prog, int32_t prog_len,
                             int32_t n_operands, int32_t n_scalars, salt_dtype dtype);

/* The cached code object (gfx950 ELF) of a compiled tree: *size gets its
 * size (0 if not compiled) and, when cap >= *size, buf a copy. */
salt_status salt_jit_code(const uint32_t *prog, int32_t prog_len, int32_t n_operands,
                          int32_t n_scalars, salt_dtype dtype, void *buf, size_t cap, size_t *size);

/* Where salt_eval would run this program now: its catalogue index (>= 0),
 * SALT_ROUTE_COMPILED when its run-time compiled kernel is ready, or -1
 * (the interpreter). No GPU work. */
salt_status salt_eval_route(const uint32_t *prog, int32_t prog_len, int32_t n_operands,
                            int32_t n_scalars, salt_dtype dtype, int32_t *route);

/* Which kernel salt_dot_expr (prog_y non-NULL) or salt_nrm2_expr (prog_y
 * NULL) runs now for these programs in `dtype`, without touching the GPU:
 * *route is the index of the pair in the library's catalogue of reduction
 * pairs with ahead-of-time kernels (dot(a + b, a - b), nrm2(a - b),
 * nrm2(alpha*a + b), with any operand and scalar numbering; a dot also with
 * its two programs exchanged), SALT_ROUTE_COMPILED when the pair's run-time
 * compiled kernel is ready, or -1 for the interpreter. All three give the
 * same bits. Programs are validated as in those calls. */
salt_status salt_reduce_expr_route(const uint32_t *prog_x, int32_t len_x,
                                   const uint32_t *prog_y, int32_t len_y,
                                   int32_t n_operands, int32_t n_scalars, salt_dtype dtype,
                                   int32_t *route);

/* Reductions of expressions (Sec. 2: a tree evaluated lazily inside a dot
 * product or a norm) whose pair is not in that catalogue run pass 1 on a
 * kernel compiled at run time for the pair, from the text of the library's
 * own pass-1 template, under the same modes and policy as trees in
 * salt_eval (SALT_JIT_AUTO: compiled at the pair's second call of at least
 * 65536 elements); pass 2 stays the library's. The cache key is the pair in
 * canonical numbering (operands and scalars numbered by first appearance in
 * prog_x, then prog_y) and the element type; a dot and the same dot with
 * its two programs exchanged share one kernel (the same bits either way).
 * Compile the pair now (blocking; needs no GPU): SALT_OK also for a pair
 * with an ahead-of-time kernel; SALT_ERR_UNSUPPORTED with the compiler's
 * log in salt_last_error() if compilation fails. */
salt_status salt_jit_compile_reduce(const uint32_t *prog_x, int32_t len_x,
                                    const uint32_t *prog_y, int32_t len_y,
                                    int32_t n_operands, int32_t n_scalars, salt_dtype dtype);

/* The cached code object (gfx950 ELF) of a compiled pair, as salt_jit_code. */
salt_status salt_jit_code_reduce(const uint32_t *prog_x, int32_t len_x,
                                 const uint32_t *prog_y, int32_t len_y,
                                 int32_t n_operands, int32_t n_scalars, salt_dtype dtype,
                                 void *buf, size_t cap, size_t *size);

/* How salt_eval launches a call of n elements of a tree that reads n_loads
 * distinct operands (no GPU work): a tree reading three or more operands,
 * over at least two chunks of 128 MiB per operand, runs as a sequence of
 * launches over contiguous chunks (the last one taking the remainder, so
 * between one and two chunks), each with the launch knobs tuned for its
 * own size; otherwise one launch. *chunk_elems gets the elements per
 * launch (n when not split), *launches the number of launches (0 for
 * n = 0). The results are the same either way. */
salt_status salt_eval_chunking(int32_t n_loads, int64_t n, salt_dtype dtype, int64_t *chunk_elems,
                               int64_t *launches);

/* Validate a program without touching the GPU. On success fills
 * *stack_need (maximum stack depth) and *n_loads (distinct operands read)
 * when those pointers are non-null. */
salt_status salt_program_check(const uint32_t *prog, int32_t prog_len,
                               int32_t n_operands, int32_t n_scalars,
                               int32_t *stack_need, int32_t *n_loads);

/* Static description of a status code; never NULL. */
const char *salt_status_string(salt_status s);

/* Thread-local detail for the last non-OK status returned on this thread
 * ("" if none). Valid until the next call on the same thread. */
const char *salt_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t salt_version(void);

/* Measurement reference, not part of the method: the plainest stream with
 * `reads` input arrays and `writes` output arrays (0 or 1) of `bytes` bytes
 * each. One 16-byte chunk per lane, no loop, integer xor of the inputs (no
 * floating point), non-temporal loads and stores. Its bandwidth for a given
 * read/write mix is what the fused-evaluation kernels are measured against
 * (a tree reading k operands and writing one result has the k-read,
 * 1-write mix). The output holds the xor of the inputs; with writes == 0
 * nothing is written and output may be NULL.
 *  reads 1..6; bytes >= 0 and a multiple of 16; inputs (host array of
 *  `reads` device pointers) and output 16-byte aligned. */
salt_status salt_stream_reference(int32_t reads, int32_t writes, const void *const *inputs,
                                  void *output, int64_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SALT_H */
