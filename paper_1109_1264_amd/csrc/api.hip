// api.hip -- the C ABI (include/salt.h): argument checks, program routing,
// launch-knob selection, and the launches themselves.
//
// This is the paper's execute function (Sec. 4.1, Fig. 2): it receives the
// tree, picks the loop (an ahead-of-time kernel for a catalogue tree, else
// the interpreter) and its unrolling (Sec. 4.3) and runs it. Every check
// happens before the first HIP call, so a rejected call has no effect.
#include <dlfcn.h>

#include <cerrno>
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <unordered_map>
#include <utility>
#include <mutex>
#include <string>
#include <vector>

#include "batch.hpp"
#include "batch_ranges.hpp"
#include "blas1.hpp"
#include "expr.hpp"
#include "jit.hpp"
#include "launch.hpp"
#include "program.hpp"
#include "salt.h"
#include "server.hpp"

namespace salt {
namespace {

thread_local std::string t_err;

salt_status fail(salt_status s, const std::string &m) {
    t_err = m;
    return s;
}

bool dtype_ok(int d) { return d >= SALT_F64 && d <= SALT_F16; }
size_t esize(int d) { return d == SALT_F64 ? 8 : d == SALT_F32 ? 4 : 2; }
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

bool partial_overlap(const void *a, const void *b, size_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    if (x == y) return false;
    return x < y + bytes && y < x + bytes;
}
bool any_overlap(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

// ---- catalogue -------------------------------------------------------------
struct CatEntry {
    int len;
    uint32_t tok[SALT_MAX_TOKENS];
    const char *name;
};

const std::vector<CatEntry> &catalogue() {
    static const std::vector<CatEntry> v = [] {
        std::vector<CatEntry> r;
        for (int id = 0; id < cat::count; ++id) {
            CatEntry e;
            e.name = "";
            e.len = catalogue_program(id, e.tok, SALT_MAX_TOKENS, &e.name);
            r.push_back(e);
        }
        return r;
    }();
    return v;
}

// Reduction pairs with ahead-of-time kernels: each entry's P and Q tokens in
// canonical numbering (expr.hpp, SALT_RCATALOGUE).
struct RcatEntry {
    int lp, lq;
    uint32_t p[SALT_MAX_TOKENS], q[SALT_MAX_TOKENS];
};

const std::vector<RcatEntry> &rcatalogue() {
    static const std::vector<RcatEntry> v = [] {
        std::vector<RcatEntry> r;
#define SALT_RCAT_EMIT(name)           \
    {                                  \
        RcatEntry e{};                 \
        rcat::name::P::emit(e.p, e.lp); \
        rcat::name::Q::emit(e.q, e.lq); \
        r.push_back(e);                \
    }
        SALT_RCATALOGUE(SALT_RCAT_EMIT)
#undef SALT_RCAT_EMIT
        return r;
    }();
    return v;
}

int route_of(const Program &p) {
    const auto &c = catalogue();
    for (size_t i = 0; i < c.size(); ++i)
        if (c[i].len == p.len && std::memcmp(c[i].tok, p.canon, sizeof(uint32_t) * p.len) == 0)
            return (int)i;
    return kRouteGeneric;
}

// ---- tuning table ------------------------------------------------------------
enum Kind { kEval = 0, kDot = 1, kNrm2 = 2, kBatch = 3 };
// Tuning-table routes: catalogue trees 0.., the interpreter -1, expression
// reductions on the interpreter -2, reduction pair id at kRouteRcat0 - id.
constexpr int kRouteRcat0 = -16;
// Run-time compiled trees (jit.hip) have their own rows under route -3.
constexpr int kRouteJit = -3;
// Bytes per operand of one launch when a large element-wise call is split
// into chunks (eval_impl).
constexpr size_t kEvalChunkBytes = (size_t)128 << 20;

// Elements per launch of an element-wise call of n elements reading n_loads
// operands: n itself, or kEvalChunkBytes per operand when the call is split
// (three or more operands and at least two chunks; the last launch takes
// the remainder, so it holds between one and two chunks).
int64_t eval_chunk_elems(int n_loads, int64_t n, int dtype) {
    const int64_t chunk = (int64_t)(kEvalChunkBytes / esize(dtype));
    return n_loads >= 3 && n >= 2 * chunk ? chunk : n;
}

struct TuneRow {
    int kind, route, dtype, log2n;
    salt_launch_config cfg;
};

// The table by (kind, route, dtype): for every log2 size the row the
// nearest-size rule picks (the first in file order among equally near
// rows), so a lookup is one hash probe instead of a scan of the table.
constexpr int kTuneSizes = 63;  // log2 n = 0 .. 62
using TuneSizes = std::array<salt_launch_config, kTuneSizes>;

uint64_t tune_key(int kind, int route, int dtype) {
    return ((uint64_t)(uint32_t)kind << 40) | ((uint64_t)(uint32_t)route << 8) | (uint64_t)(uint8_t)dtype;
}

std::unordered_map<uint64_t, TuneSizes> index_tune(const std::vector<TuneRow> &rows) {
    std::unordered_map<uint64_t, TuneSizes> ix;
    std::unordered_map<uint64_t, std::array<int, kTuneSizes>> dist;
    for (const TuneRow &r : rows) {
        const uint64_t k = tune_key(r.kind, r.route, r.dtype);
        auto d = dist.try_emplace(k);
        if (d.second) d.first->second.fill(INT_MAX);
        TuneSizes &cfgs = ix[k];
        for (int l = 0; l < kTuneSizes; ++l) {
            const int dl = std::abs(r.log2n - l);
            if (dl < d.first->second[l]) {
                d.first->second[l] = dl;
                cfgs[l] = r.cfg;
            }
        }
    }
    return ix;
}

std::mutex g_tune_mu;
std::unordered_map<uint64_t, TuneSizes> g_tune;  // the loaded table, indexed
bool g_tune_loaded = false;

std::string default_tune_path() {
    if (const char *e = std::getenv("SALT_TUNE_FILE")) return e;
    Dl_info info;
    if (dladdr((void *)&salt_version, &info) && info.dli_fname) {
        std::string f = info.dli_fname;
        const size_t slash = f.rfind('/');
        return (slash == std::string::npos ? std::string(".") : f.substr(0, slash)) + "/salt_tuning.txt";
    }
    return "salt_tuning.txt";
}

bool parse_tune(const std::string &path, std::vector<TuneRow> &rows, std::string *why) {
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) {
        if (why) *why = "cannot open tuning file " + path;
        return false;
    }
    char line[256];
    int lineno = 0;
    bool ok = true;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        char *h = std::strchr(line, '#');
        if (h) *h = 0;
        char kind[16];
        int route, dtype, log2n, unroll, nt;
        long long blocks;
        int got = std::sscanf(line, "%15s %d %d %d %d %d %lld", kind, &route, &dtype, &log2n, &unroll, &nt, &blocks);
        if (got <= 0) continue;
        TuneRow r;
        r.kind = !std::strcmp(kind, "eval") ? kEval : !std::strcmp(kind, "dot") ? kDot
               : !std::strcmp(kind, "nrm2") ? kNrm2 : !std::strcmp(kind, "batch") ? kBatch : -1;
        if (got != 7 || r.kind < 0 || !dtype_ok(dtype) || log2n < 0 || log2n > 62 || nt < 0 || nt > 1 || blocks < 0) {
            if (why) *why = path + ": bad row at line " + std::to_string(lineno);
            ok = false;
            break;
        }
        r.route = route;
        r.dtype = dtype;
        r.log2n = log2n;
        r.cfg.unroll = unroll;
        r.cfg.nontemporal = nt;
        r.cfg.blocks = blocks;
        rows.push_back(r);
    }
    std::fclose(f);
    return ok;
}

void ensure_tune_loaded() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::vector<TuneRow> rows;
    if (parse_tune(default_tune_path(), rows, nullptr)) g_tune = index_tune(rows);
}

int ilog2(int64_t n) { return n > 1 ? 63 - __builtin_clzll((unsigned long long)n) : 0; }

// Defaults before any measurement: 4 chunks per operand per lane, streaming
// hints above the 256 MiB last-level cache, one workgroup per tile.
salt_launch_config default_cfg(int kind, int dtype, int64_t n, int n_arrays) {
    salt_launch_config c;
    const double bytes = (double)n * (double)esize(dtype) * n_arrays;
    c.unroll = kind == kEval ? 4 : 8;
    if (kind == kEval && bytes >= 256.0 * 1024 * 1024) c.unroll = n_arrays <= 3 ? 1 : 4;
    c.nontemporal = bytes >= 256.0 * 1024 * 1024 ? 1 : 0;
    c.blocks = 0;
    return c;
}

salt_launch_config lookup(int kind, int route, int dtype, int64_t n, int n_arrays) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    ensure_tune_loaded();
    const auto it = g_tune.find(tune_key(kind, route, dtype));
    if (it == g_tune.end()) return default_cfg(kind, dtype, n, n_arrays);
    return it->second[std::min(ilog2(n > 0 ? n : 1), kTuneSizes - 1)];
}

// Knobs of a call: the tuned values, overridden by the caller's. Unroll
// values: eval 1, 2, 4, 8; dot / nrm2 2, 4, 8, 16; batched 2, 4, 8.
salt_status resolve(const salt_launch_config *req, salt_launch_config tuned, int kind,
                    salt_launch_config *out) {
    salt_launch_config c = tuned;
    if (req) {
        if (req->unroll != 0) c.unroll = req->unroll;
        if (req->nontemporal >= 0) c.nontemporal = req->nontemporal;
        if (req->blocks >= 0) c.blocks = req->blocks;
        if (req->nontemporal > 1 || req->blocks < -1 || req->nontemporal < -1)
            return fail(SALT_ERR_ARG, "launch config out of range");
    }
    const int u = c.unroll;
    const bool ok = kind == kEval ? (u == 1 || u == 2 || u == 4 || u == 8)
                  : kind == kBatch ? (u == 2 || u == 4 || u == 8)
                  : (u == 2 || u == 4 || u == 8 || u == 16);
    if (!ok) return fail(SALT_ERR_ARG, "unroll " + std::to_string(u) + " not available");
    *out = c;
    return SALT_OK;
}

salt_status device_status(hipError_t e) {
    if (e == hipSuccess) return SALT_OK;
    return fail(SALT_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
}

salt_status eval_impl(const uint32_t *prog, int32_t prog_len, const void *const *operands,
                      int32_t n_operands, const double *scalars, int32_t n_scalars, void *out,
                      int64_t n, int dtype, void *stream, const salt_launch_config *cfg) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    if ((uint64_t)n > (uint64_t)INT64_MAX / 16) return fail(SALT_ERR_ARG, "length too large");
    Program p;
    std::string why;
    salt_status s = compile_program(prog, prog_len, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, why);
    if (p.n_loads > 0 && !operands) return fail(SALT_ERR_ARG, "operand array is NULL");
    if (p.n_scal > 0 && !scalars) return fail(SALT_ERR_ARG, "scalar array is NULL");
    const int route = route_of(p);
    salt_launch_config c;  // checks the caller's knobs before anything runs (each launch resolves its own)
    s = resolve(cfg, lookup(kEval, route, dtype, n, p.n_loads + 1), kEval, &c);
    if (s != SALT_OK) return s;
    if (n == 0) return SALT_OK;
    if (!out) return fail(SALT_ERR_ARG, "output pointer is NULL");

    EvalLaunch L;
    std::memset(&L, 0, sizeof L);
    const size_t es = esize(dtype);
    const size_t bytes = (size_t)n * es;
    bool vec = aligned16(out);
    for (int k = 0; k < p.n_loads; ++k) {
        const void *a = operands[p.op_map[k]];
        if (!a) return fail(SALT_ERR_ARG, "operand " + std::to_string(p.op_map[k]) + " is NULL");
        if (partial_overlap(a, out, bytes))
            return fail(SALT_ERR_ARG, "output partially overlaps operand " + std::to_string(p.op_map[k]));
        L.ops[k] = a;
        vec = vec && aligned16(a);
    }
    for (int j = 0; j < p.n_scal; ++j) L.sc[j] = scalars[p.sc_map[j]];
    L.vec = vec ? 1 : 0;
    L.stream = stream;
    EvalFn fn = nullptr;
    if (route != kRouteGeneric) {
        fn = catalogue_launcher(route, dtype);
        if (!fn) return fail(SALT_ERR_UNSUPPORTED, "no kernel for this tree and dtype");
    }
    // Elements [off, off + m) as one launch, with the knobs tuned for m. A
    // tree outside the catalogue runs its run-time compiled kernel when it
    // is ready (with the compiled kernels' own tuned knobs), else the
    // interpreter (same bits either way).
    bool try_jit = route == kRouteGeneric && jit_mode() != kJitOff;
    const auto launch_range = [&](int64_t off, int64_t m) -> salt_status {
        EvalLaunch R = L;
        for (int k = 0; k < p.n_loads; ++k) R.ops[k] = (const char *)L.ops[k] + (size_t)off * es;
        R.out = (char *)out + (size_t)off * es;
        R.n = m;
        salt_launch_config cr;
        salt_status st = resolve(cfg, lookup(kEval, route, dtype, m, p.n_loads + 1), kEval, &cr);
        if (st != SALT_OK) return st;
        R.unroll = cr.unroll;
        R.nontemporal = cr.nontemporal;
        R.blocks = cr.blocks;
        if (fn) return device_status(fn(R));
        if (try_jit) {
            salt_launch_config cj;
            st = resolve(cfg, lookup(kEval, kRouteJit, dtype, m, p.n_loads + 1), kEval, &cj);
            if (st != SALT_OK) return st;
            EvalLaunch RJ = R;
            RJ.unroll = cj.unroll;
            RJ.nontemporal = cj.nontemporal;
            RJ.blocks = cj.blocks;
            bool ran = false;
            const hipError_t je = jit_try_launch(RJ, p, dtype, &ran);
            if (ran || je != hipSuccess) return device_status(je);
            try_jit = false;  // a call that started interpreted stays so (one step of the policy per call)
        }
        return device_status(launch_interp(R, p, dtype));
    };
    // A large call of a tree that reads three or more operands runs as a
    // sequence of launches over contiguous chunks (kEvalChunkBytes per
    // operand, the last one taking the remainder), each with the knobs of
    // its own size. The persistent grid those knobs choose then restarts in
    // step at every chunk instead of drifting apart over the whole array;
    // measured 4-14 % faster for five or six operands at 2 GiB per operand,
    // and no faster for one or two. Each element is computed exactly as in
    // one launch.
    const int64_t chunk = eval_chunk_elems(p.n_loads, n, dtype);
    if (chunk < n) {
        const int64_t parts = n / chunk;
        for (int64_t q = 0; q < parts; ++q) {
            const int64_t off = q * chunk;
            s = launch_range(off, q + 1 < parts ? chunk : n - off);
            if (s != SALT_OK) return s;
        }
        return SALT_OK;
    }
    return launch_range(0, n);
}

// dot (mode kModeDot) reads x and y; nrm2 and asum read x only and share
// nrm2's tuning (the same traffic).
salt_status reduce_impl(int64_t n, const void *x, const void *y, void *result, void *ws,
                        size_t ws_bytes, int dtype, void *stream, const salt_launch_config *cfg,
                        int mode) {
    const bool nrm2 = mode != kModeDot;  // one operand
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    if ((uint64_t)n > (uint64_t)INT64_MAX / 16) return fail(SALT_ERR_ARG, "length too large");
    if (!result) return fail(SALT_ERR_ARG, "result pointer is NULL");
    if (n > 0 && (!x || (!nrm2 && !y))) return fail(SALT_ERR_ARG, "input pointer is NULL");
    const size_t need = salt_reduce_workspace_bytes(n, (salt_dtype)dtype);
    if (need > 0) {
        if (!ws) return fail(SALT_ERR_WORKSPACE, "workspace is NULL");
        if (((uintptr_t)ws & 7u) != 0) return fail(SALT_ERR_WORKSPACE, "workspace not 8-byte aligned");
        if (ws_bytes < need)
            return fail(SALT_ERR_WORKSPACE, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                                std::to_string(need));
        const size_t bytes = (size_t)n * esize(dtype);
        if (any_overlap(ws, need, x, bytes) || (!nrm2 && any_overlap(ws, need, y, bytes)))
            return fail(SALT_ERR_WORKSPACE, "workspace overlaps an input");
    }
    salt_launch_config c;
    salt_status s = resolve(cfg, lookup(nrm2 ? kNrm2 : kDot, -1, dtype, n, nrm2 ? 1 : 2), nrm2 ? kNrm2 : kDot, &c);
    if (s != SALT_OK) return s;
    ReduceLaunch L;
    L.x = x;
    L.y = nrm2 ? x : y;
    L.result = result;
    L.ws = (double *)ws;
    L.n = n;
    L.vec = aligned16(x) && (nrm2 || aligned16(y)) ? 1 : 0;
    L.unroll = c.unroll;
    L.nontemporal = c.nontemporal;
    L.blocks = c.blocks;
    L.mode = mode;
    L.passes = 3;
    L.n_partials = 0;
    L.stream = stream;
    return device_status(launch_reduce(L, dtype));
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- BLAS level-1 with increments -----------------------------------------
constexpr int64_t kMaxSpan = (int64_t)1 << 59;  // elements one strided vector may span

uint64_t abs_inc(int64_t inc) { return inc < 0 ? (uint64_t)(-(inc + 1)) + 1u : (uint64_t)inc; }

// Bytes from the vector's pointer to the end of its last element.
size_t span_bytes(int64_t n, int64_t inc, int dtype) {
    return n <= 0 ? 0 : (size_t)(1 + (uint64_t)(n - 1) * abs_inc(inc)) * esize(dtype);
}

salt_status check_vec(int64_t n, const void *p, int64_t inc, const char *name, bool output) {
    if (n <= 0) return SALT_OK;
    if (!p) return fail(SALT_ERR_ARG, std::string(name) + " is NULL");
    if (n > 1 && abs_inc(inc) > (uint64_t)(kMaxSpan - 1) / (uint64_t)(n - 1))
        return fail(SALT_ERR_ARG, std::string(name) + ": the strided vector spans more than 2^59 elements");
    if (output && inc == 0 && n > 1)
        return fail(SALT_ERR_ARG, std::string(name) + ": output increment 0 would write one element n times");
    return SALT_OK;
}

salt_status check_reduce_ws(int64_t n, int dtype, void *ws, size_t ws_bytes, const void *x, size_t xb,
                            const void *y, size_t yb) {
    const size_t need = salt_reduce_workspace_bytes(n, (salt_dtype)dtype);
    if (need == 0) return SALT_OK;
    if (!ws) return fail(SALT_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 7u) != 0) return fail(SALT_ERR_WORKSPACE, "workspace not 8-byte aligned");
    if (ws_bytes < need)
        return fail(SALT_ERR_WORKSPACE,
                    "workspace has " + std::to_string(ws_bytes) + " bytes, needs " + std::to_string(need));
    if (any_overlap(ws, need, x, xb) || (y && any_overlap(ws, need, y, yb)))
        return fail(SALT_ERR_WORKSPACE, "workspace overlaps an input");
    return SALT_OK;
}

// dot (both vectors), nrm2 / asum (x only; inc <= 0 gives 0 as in BLAS).
salt_status strided_reduce_impl(int64_t n, const void *x, int64_t incx, const void *y, int64_t incy,
                                void *result, void *ws, size_t ws_bytes, int dtype, void *stream, int mode) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    if (!result) return fail(SALT_ERR_ARG, "result pointer is NULL");
    const bool dot = mode == kModeDot;
    if (!dot && incx <= 0) n = 0;
    salt_status s = check_vec(n, x, incx, "x", false);
    if (s == SALT_OK && dot) s = check_vec(n, y, incy, "y", false);
    if (s != SALT_OK) return s;
    if (n == 0 || (incx == 1 && (!dot || incy == 1)))
        return reduce_impl(n, x, dot ? y : x, result, ws, ws_bytes, dtype, stream, nullptr, mode);
    s = check_reduce_ws(n, dtype, ws, ws_bytes, x, span_bytes(n, incx, dtype), dot ? y : nullptr,
                        dot ? span_bytes(n, incy, dtype) : 0);
    if (s != SALT_OK) return s;
    StridedReduceLaunch L;
    L.x = x;
    L.incx = incx;
    L.y = dot ? y : x;
    L.incy = dot ? incy : incx;
    L.result = result;
    L.ws = (double *)ws;
    L.n = n;
    L.mode = mode;
    L.stream = stream;
    return device_status(launch_strided_reduce(L, dtype));
}

}  // namespace
}  // namespace salt

struct salt_batch_plan_s {
    int route = -1, dtype = 0, count = 0;  // route: catalogue id, or -3 (compiled at run time)
    salt::Program prog;                    // the tree, canonical (for a compiled route)
    int64_t total_tiles = 0, total_elems = 0;
    bool any_dot = false;
    std::vector<salt::DevItem> items;
    std::vector<salt::TileRef> tiles;
    size_t table_bytes = 0, ws_bytes = 0;
    void *table = nullptr;
};

struct salt_graph_s {
    hipGraphExec_t exec = nullptr;
};

using namespace salt;

namespace salt {
namespace {

salt_status batch_launch_impl(salt_batch_plan plan, void *ws, size_t ws_bytes, void *stream,
                              const salt_launch_config *cfg) {
    if (!plan) return fail(SALT_ERR_ARG, "plan is NULL");
    if (!plan->table) return fail(SALT_ERR_ARG, "plan has not been uploaded");
    if (plan->ws_bytes > 0) {
        if (!ws) return fail(SALT_ERR_WORKSPACE, "workspace is NULL");
        if (((uintptr_t)ws & 7u) != 0) return fail(SALT_ERR_WORKSPACE, "workspace not 8-byte aligned");
        if (ws_bytes < plan->ws_bytes) return fail(SALT_ERR_WORKSPACE, "workspace too small");
    }
    salt_launch_config c;
    salt_status s = resolve(cfg, lookup(kBatch, plan->route, plan->dtype, plan->total_elems, 4), kBatch, &c);
    if (s != SALT_OK) return s;
    if (plan->count == 0) return SALT_OK;
    BatchFn fn = nullptr;
    if (plan->route != kRouteJit) {
        fn = catalogue_batch_launcher(plan->route, plan->dtype);
        if (!fn) return fail(SALT_ERR_UNSUPPORTED, "no batched kernel for this tree and dtype");
    }
    BatchLaunch L;
    L.items = (const DevItem *)plan->table;
    L.tiles = (const TileRef *)((const char *)plan->table + sizeof(DevItem) * plan->count);
    L.total_tiles = plan->total_tiles;
    L.count = plan->count;
    L.any_dot = plan->any_dot ? 1 : 0;
    L.ws = (double *)ws;
    L.unroll = c.unroll;
    L.nontemporal = c.nontemporal;
    L.blocks = c.blocks;
    L.stream = stream;
    L.combine = 1;
    // a long execution list runs as several launches over consecutive ranges
    // (batch_ranges.hpp), each with the knobs tuned for its size
    const auto knobs = [&](int64_t elems, BatchLaunch &r) -> int {
        salt_launch_config k;
        if (resolve(cfg, lookup(kBatch, plan->route, plan->dtype, elems, 4), kBatch, &k) != SALT_OK)
            return (int)hipErrorInvalidValue;
        r.unroll = k.unroll;
        r.nontemporal = k.nontemporal;
        r.blocks = k.blocks;
        return 0;
    };
    const auto launch = [&](const BatchLaunch &r) -> int {
        return plan->route == kRouteJit ? (int)jit_batch_launch(r, plan->prog, plan->dtype) : fn(r);
    };
    return device_status((hipError_t)launch_batch_ranges(launch, L, plan->total_elems, reduce_tile_elems(plan->dtype),
                                                         (int64_t)esize(plan->dtype), knobs));
}

int canon_pair(const uint32_t *a, int32_t la, const uint32_t *b, int32_t lb, uint32_t *ca, uint32_t *cb,
               int32_t *op_map, int32_t *sc_map);

// The pair (P, Q) (Q null: nrm2(P)) of validated programs in canonical
// numbering, for the run-time compiler; op_map / sc_map as canon_pair's. A
// dot takes whichever order of its two programs gives the smaller canonical
// form (the product is symmetric, so both orders give the same bits), so
// dot(P, Q) and dot(Q, P) share one compiled kernel.
PairTrees pair_trees(const uint32_t *px, int32_t lx, const uint32_t *py, int32_t ly, int32_t *op_map,
                     int32_t *sc_map, int *n_scalars) {
    const auto one = [](const uint32_t *a, int32_t la, const uint32_t *b, int32_t lb, bool nrm2, int32_t *om,
                        int32_t *sm, int *ns) {
        PairTrees t;
        t.nrm2 = nrm2;
        t.lp = la;
        t.lq = lb;
        for (int k = 0; k < SALT_MAX_OPERANDS; ++k) om[k] = -1;
        *ns = canon_pair(a, la, b, lb, t.p, t.q, om, sm);
        t.n_loads = 0;
        while (t.n_loads < SALT_MAX_OPERANDS && om[t.n_loads] >= 0) ++t.n_loads;
        return t;
    };
    int ns = 0;
    PairTrees t = one(px, lx, py, py ? ly : 0, py == nullptr, op_map, sc_map, &ns);
    if (py) {
        int32_t om2[SALT_MAX_OPERANDS], sm2[SALT_MAX_SCALARS];
        int ns2 = 0;
        const PairTrees u = one(py, ly, px, lx, false, om2, sm2, &ns2);
        const auto form = [](const PairTrees &v) {
            std::vector<uint32_t> f(v.p, v.p + v.lp);
            f.push_back(0xffffffffu);  // no token has this value: separates P from Q
            f.insert(f.end(), v.q, v.q + v.lq);
            return f;
        };
        if (form(u) < form(t)) {
            t = u;
            ns = ns2;
            std::memcpy(op_map, om2, sizeof om2);
            std::memcpy(sc_map, sm2, sizeof sm2);
        }
    }
    if (n_scalars) *n_scalars = ns;
    return t;
}

salt_status reduce_expr_impl(const uint32_t *px, int32_t lx, const uint32_t *py, int32_t ly,
                             const void *const *operands, int32_t n_operands, const double *scalars,
                             int32_t n_scalars, int64_t n, void *result, void *ws, size_t ws_bytes, int dtype,
                             void *stream, bool nrm2, const salt_launch_config *cfg) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    if ((uint64_t)n > (uint64_t)INT64_MAX / 16) return fail(SALT_ERR_ARG, "length too large");
    Program gx, gy;
    std::string why;
    salt_status s = compile_program(px, lx, n_operands, n_scalars, &gx, &why);
    if (s != SALT_OK) return fail(s, "first program: " + why);
    if (!nrm2) {
        s = compile_program(py, ly, n_operands, n_scalars, &gy, &why);
        if (s != SALT_OK) return fail(s, "second program: " + why);
    }
    // The second program runs one stack slot up, on the first one's result.
    if (!nrm2 && gy.stack_need > SALT_MAX_STACK - 1) {
        if (gx.stack_need <= SALT_MAX_STACK - 1) std::swap(gx, gy);  // the product is symmetric
        else return fail(SALT_ERR_UNSUPPORTED, "both programs need all 8 stack slots");
    }
    const uint32_t mask = gx.load_mask | (nrm2 ? 0u : gy.load_mask);
    if (mask && !operands) return fail(SALT_ERR_ARG, "operand array is NULL");
    if ((gx.n_scal || (!nrm2 && gy.n_scal)) && !scalars) return fail(SALT_ERR_ARG, "scalar array is NULL");
    if (!result) return fail(SALT_ERR_ARG, "result pointer is NULL");
    ReduceExprLaunch L;
    std::memset(&L, 0, sizeof L);
    const size_t bytes = (size_t)n * esize(dtype);
    const size_t need = salt_reduce_workspace_bytes(n, (salt_dtype)dtype);
    bool vec = true;
    for (int k = 0; k < SALT_MAX_OPERANDS; ++k) {
        if (!((mask >> k) & 1u)) continue;
        if (n > 0 && !operands[k]) return fail(SALT_ERR_ARG, "operand " + std::to_string(k) + " is NULL");
        if (need > 0 && any_overlap(ws, need, operands[k], bytes))
            return fail(SALT_ERR_WORKSPACE, "workspace overlaps an operand");
        L.ops[k] = operands[k];
        vec = vec && aligned16(operands[k]);
    }
    if (need > 0) {
        if (!ws) return fail(SALT_ERR_WORKSPACE, "workspace is NULL");
        if (((uintptr_t)ws & 7u) != 0) return fail(SALT_ERR_WORKSPACE, "workspace not 8-byte aligned");
        if (ws_bytes < need) return fail(SALT_ERR_WORKSPACE, "workspace too small");
    }
    for (int j = 0; j < n_scalars && j < SALT_MAX_SCALARS; ++j) L.sc[j] = scalars ? scalars[j] : 0.0;
    // A pair with an ahead-of-time kernel runs it (same bits as the
    // interpreter); its tuned knobs live under route kRouteRcat0 - id.
    int32_t om[SALT_MAX_OPERANDS], sm[SALT_MAX_SCALARS], nsc = 0;
    const int rid = route_pair(px, lx, nrm2 ? nullptr : py, nrm2 ? 0 : ly, om, sm, &nsc);
    salt_launch_config c;
    if (rid >= 0) {
        int nl = 0;
        for (int k = 0; k < SALT_MAX_OPERANDS; ++k) nl += (mask >> k) & 1u;
        s = resolve(cfg, lookup(nrm2 ? kNrm2 : kDot, kRouteRcat0 - rid, dtype, n, nl), nrm2 ? kNrm2 : kDot, &c);
        if (s != SALT_OK) return s;
        ReduceExprLaunch R;
        std::memset(&R, 0, sizeof R);
        for (int k = 0; k < nl; ++k) R.ops[k] = operands[om[k]];
        for (int j = 0; j < nsc && j < SALT_MAX_SCALARS; ++j) R.sc[j] = scalars[sm[j]];
        R.result = result;
        R.ws = (double *)ws;
        R.n = n;
        R.vec = vec ? 1 : 0;
        R.unroll = c.unroll;
        R.nontemporal = c.nontemporal;
        R.blocks = c.blocks;
        R.nrm2 = nrm2 ? 1 : 0;
        R.stream = stream;
        return device_status(launch_reduce_tree(R, rid, dtype));
    }
    // Any other pair: pass 1 on its run-time compiled kernel when that is
    // ready (knobs under route kRouteJit), with the library's pass 2; the
    // interpreter otherwise. Same bits either way.
    if (jit_mode() != kJitOff && n > 0) {
        int32_t jm[SALT_MAX_OPERANDS], js[SALT_MAX_SCALARS];
        int jns = 0;
        const PairTrees t = pair_trees(px, lx, nrm2 ? nullptr : py, nrm2 ? 0 : ly, jm, js, &jns);
        salt_launch_config cj;
        s = resolve(cfg, lookup(nrm2 ? kNrm2 : kDot, kRouteJit, dtype, n, t.n_loads), nrm2 ? kNrm2 : kDot, &cj);
        if (s != SALT_OK) return s;
        ReduceExprLaunch R;
        std::memset(&R, 0, sizeof R);
        for (int k = 0; k < t.n_loads; ++k) R.ops[k] = operands[jm[k]];
        for (int j = 0; j < jns && j < SALT_MAX_SCALARS; ++j) R.sc[j] = scalars[js[j]];
        R.result = result;
        R.ws = (double *)ws;
        R.n = n;
        R.vec = vec ? 1 : 0;
        R.unroll = cj.unroll;
        R.nontemporal = cj.nontemporal;
        R.blocks = cj.blocks;
        R.nrm2 = nrm2 ? 1 : 0;
        R.stream = stream;
        bool ran = false;
        const hipError_t je = jit_try_reduce(R, t, dtype, &ran);
        if (je != hipSuccess) return device_status(je);
        if (ran) {
            const int64_t T = reduce_tile_elems(dtype);
            const int64_t n_tiles = (n + T - 1) / T;
            if (n_tiles == 1) return SALT_OK;  // pass 1 stored the result
            ReduceLaunch P2;
            std::memset(&P2, 0, sizeof P2);
            P2.result = result;
            P2.ws = (double *)ws;
            P2.n = n;
            P2.mode = nrm2 ? kModeNrm2 : kModeDot;
            P2.passes = 2;
            P2.n_partials = n_tiles;
            P2.stream = stream;
            return device_status(launch_reduce(P2, dtype));
        }
    }
    // Tuned knobs of the expression reductions on the interpreter live under
    // route -2.
    s = resolve(cfg, lookup(nrm2 ? kNrm2 : kDot, -2, dtype, n, nrm2 ? 1 : 2), nrm2 ? kNrm2 : kDot, &c);
    if (s != SALT_OK) return s;
    L.result = result;
    L.unroll = c.unroll;
    L.ws = (double *)ws;
    L.n = n;
    L.vec = vec ? 1 : 0;
    L.mask = mask;
    L.nontemporal = c.nontemporal;
    L.blocks = c.blocks;
    L.nrm2 = nrm2 ? 1 : 0;
    L.stream = stream;
    return device_status(launch_reduce_expr(L, gx, nrm2 ? nullptr : &gy, dtype));
}

// Canonical numbering over the concatenation of two validated programs:
// operands and scalars numbered by first appearance in a, then in b.
// Returns the number of distinct scalars read.
int canon_pair(const uint32_t *a, int32_t la, const uint32_t *b, int32_t lb, uint32_t *ca, uint32_t *cb,
               int32_t *op_map, int32_t *sc_map) {
    int32_t opn[SALT_MAX_OPERANDS], scn[SALT_MAX_SCALARS];
    for (auto &x : opn) x = -1;
    for (auto &x : scn) x = -1;
    int no = 0, ns = 0;
    const auto one = [&](uint32_t t) -> uint32_t {
        const uint32_t op = t & 0xffu, arg = t >> 8;
        if (op == SALT_OP_LOAD) {
            if (opn[arg] < 0) op_map[no] = (int32_t)arg, opn[arg] = no++;
            return SALT_TOKEN(SALT_OP_LOAD, opn[arg]);
        }
        if (op == SALT_OP_SCALAR) {
            if (scn[arg] < 0) sc_map[ns] = (int32_t)arg, scn[arg] = ns++;
            return SALT_TOKEN(SALT_OP_SCALAR, scn[arg]);
        }
        return t;
    };
    for (int i = 0; i < la; ++i) ca[i] = one(a[i]);
    for (int i = 0; i < lb; ++i) cb[i] = one(b[i]);
    return ns;
}

}  // namespace

int route_pair(const uint32_t *px, int32_t lx, const uint32_t *py, int32_t ly, int32_t *op_map,
               int32_t *sc_map, int32_t *n_scalars) {
    const auto &cat = rcatalogue();
    for (int order = 0; order < (py ? 2 : 1); ++order) {
        const uint32_t *a = order ? py : px, *b = order ? px : py;
        const int32_t la = order ? ly : lx, lb = py ? (order ? lx : ly) : 0;
        uint32_t ca[SALT_MAX_TOKENS], cb[SALT_MAX_TOKENS];
        int32_t om[SALT_MAX_OPERANDS], sm[SALT_MAX_SCALARS];
        const int ns = canon_pair(a, la, b, lb, ca, cb, om, sm);
        for (size_t id = 0; id < cat.size(); ++id) {
            const RcatEntry &e = cat[id];
            if (e.lp != la || e.lq != lb) continue;
            if (std::memcmp(e.p, ca, sizeof(uint32_t) * la) || std::memcmp(e.q, cb, sizeof(uint32_t) * lb)) continue;
            std::memcpy(op_map, om, sizeof om);
            std::memcpy(sc_map, sm, sizeof sm);
            if (n_scalars) *n_scalars = ns;
            return (int)id;
        }
    }
    return -1;
}

salt_status tuned_config(int kind, int route, int dtype, int64_t n, salt_launch_config *out) {
    if (!out || !dtype_ok(dtype)) return SALT_ERR_ARG;
    *out = lookup(kind, route, dtype, n, kind == kNrm2 ? 1 : kind == kBatch ? 4 : 2);
    return SALT_OK;
}

// Validate the programs of a dot (prog_y non-null) or nrm2 of expressions,
// with the rule the reduction applies: one of a dot's two programs must fit
// in SALT_MAX_STACK - 1 slots.
salt_status check_pair(const uint32_t *prog_x, int32_t len_x, const uint32_t *prog_y, int32_t len_y,
                       int32_t n_operands, int32_t n_scalars) {
    Program p, q;
    std::string why;
    salt_status s = compile_program(prog_x, len_x, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, "first program: " + why);
    if (prog_y) {
        s = compile_program(prog_y, len_y, n_operands, n_scalars, &q, &why);
        if (s != SALT_OK) return fail(s, "second program: " + why);
        if (p.stack_need > SALT_MAX_STACK - 1 && q.stack_need > SALT_MAX_STACK - 1)
            return fail(SALT_ERR_UNSUPPORTED, "both programs need all 8 stack slots");
    }
    return SALT_OK;
}


}  // namespace salt

// ---- dot without a caller workspace -----------------------------------------
// The tile partials of salt_dot_noalloc live in this file-scope array, one
// copy per GPU, for the life of the process. Host code never passes the
// array's name to a kernel (on the host it is only a stand-in): the device
// address of each GPU's copy is looked up once, with that GPU current, and
// that address is what the launches receive.
namespace salt {
constexpr int64_t kNoallocPartials = SALT_NOALLOC_MAX_PARTIALS;
static __device__ __align__(256) double scratch[kNoallocPartials];

namespace {
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's `scratch`, looked up on first use.
salt_status scratch_for_current_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SALT_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SALT_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SALT_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SALT_OK;
}
}  // namespace
}  // namespace salt

extern "C" {

salt_status salt_eval(const uint32_t *prog, int32_t prog_len, const void *const *operands,
                      int32_t n_operands, const double *scalars, int32_t n_scalars, void *out,
                      int64_t n, salt_dtype dtype, void *hip_stream) {
    return eval_impl(prog, prog_len, operands, n_operands, scalars, n_scalars, out, n, dtype, hip_stream,
                     nullptr);
}

salt_status salt_eval_ex(const uint32_t *prog, int32_t prog_len, const void *const *operands,
                         int32_t n_operands, const double *scalars, int32_t n_scalars, void *out,
                         int64_t n, salt_dtype dtype, void *hip_stream, const salt_launch_config *cfg) {
    return eval_impl(prog, prog_len, operands, n_operands, scalars, n_scalars, out, n, dtype, hip_stream,
                     cfg);
}

salt_status salt_axpy(int64_t n, double alpha, const void *x, void *y, salt_dtype dtype, void *hip_stream) {
    static const uint32_t prog[5] = {SALT_TOKEN(SALT_OP_SCALAR, 0), SALT_TOKEN(SALT_OP_LOAD, 0),
                                     SALT_TOKEN(SALT_OP_MUL, 0), SALT_TOKEN(SALT_OP_LOAD, 1),
                                     SALT_TOKEN(SALT_OP_ADD, 0)};
    if (n > 0 && dtype_ok(dtype) && x && y && x != y &&
        any_overlap(x, (size_t)n * esize(dtype), y, (size_t)n * esize(dtype)))
        return fail(SALT_ERR_ARG, "x partially overlaps y");
    const void *ops[2] = {x, y};
    return eval_impl(prog, 5, ops, 2, &alpha, 1, y, n, dtype, hip_stream, nullptr);
}

size_t salt_reduce_workspace_bytes(int64_t n, salt_dtype dtype) {
    const int64_t T = reduce_tile_elems(dtype);
    if (n <= 0 || T <= 0) return 0;
    return (size_t)((n + T - 1) / T) * sizeof(double);
}

int64_t salt_reduce_tile_elems(salt_dtype dtype) { return reduce_tile_elems(dtype); }

salt_status salt_dot(int64_t n, const void *x, const void *y, void *result, void *workspace,
                     size_t ws_bytes, salt_dtype dtype, void *hip_stream) {
    return reduce_impl(n, x, y, result, workspace, ws_bytes, dtype, hip_stream, nullptr, kModeDot);
}

salt_status salt_dot_noalloc(int64_t n, const void *x, const void *y, void *result, salt_dtype dtype,
                             void *hip_stream) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    const size_t need = salt_reduce_workspace_bytes(n, dtype);
    if (need > (size_t)kNoallocPartials * sizeof(double))
        return fail(SALT_ERR_UNSUPPORTED, "n = " + std::to_string(n) + " needs " + std::to_string(need / 8) +
                                              " tile partials; the built-in buffer holds " +
                                              std::to_string(kNoallocPartials));
    void *ws = nullptr;
    if (need > 0) {
        // argument errors first, so a rejected call touches no HIP state
        if (!result) return fail(SALT_ERR_ARG, "result pointer is NULL");
        if (!x || !y) return fail(SALT_ERR_ARG, "input pointer is NULL");
        salt_status s = scratch_for_current_device(&ws);
        if (s != SALT_OK) return s;
    }
    return reduce_impl(n, x, y, result, ws, need, dtype, hip_stream, nullptr, kModeDot);
}

salt_status salt_dot_ex(int64_t n, const void *x, const void *y, void *result, void *workspace,
                        size_t ws_bytes, salt_dtype dtype, void *hip_stream, const salt_launch_config *cfg) {
    return reduce_impl(n, x, y, result, workspace, ws_bytes, dtype, hip_stream, cfg, kModeDot);
}

salt_status salt_reduce_partials(int32_t mode, int64_t n, const void *x, const void *y, double *partials,
                                 salt_dtype dtype, void *hip_stream) {
    if (mode < kModeDot || mode > kModeAsum) return fail(SALT_ERR_ARG, "mode " + std::to_string(mode) + " outside 0..2");
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    if ((uint64_t)n > (uint64_t)INT64_MAX / 16) return fail(SALT_ERR_ARG, "length too large");
    const bool two = mode == kModeDot;
    if (n == 0) return SALT_OK;  // no tiles, no partials
    if (!x || (two && !y)) return fail(SALT_ERR_ARG, "input pointer is NULL");
    if (!partials) return fail(SALT_ERR_ARG, "partials pointer is NULL");
    if (((uintptr_t)partials & 7u) != 0) return fail(SALT_ERR_ARG, "partials not 8-byte aligned");
    const size_t need = salt_reduce_workspace_bytes(n, dtype), bytes = (size_t)n * esize(dtype);
    if (any_overlap(partials, need, x, bytes) || (two && any_overlap(partials, need, y, bytes)))
        return fail(SALT_ERR_ARG, "partials overlap an input");
    salt_launch_config c;
    salt_status s = resolve(nullptr, lookup(two ? kDot : kNrm2, -1, dtype, n, two ? 2 : 1), two ? kDot : kNrm2, &c);
    if (s != SALT_OK) return s;
    ReduceLaunch L;
    L.x = x;
    L.y = two ? y : x;
    L.result = nullptr;
    L.ws = partials;
    L.n = n;
    L.vec = aligned16(x) && (!two || aligned16(y)) ? 1 : 0;
    L.unroll = c.unroll;
    L.nontemporal = c.nontemporal;
    L.blocks = c.blocks;
    L.mode = mode;
    L.passes = 1;
    L.n_partials = 0;
    L.stream = hip_stream;
    return device_status(launch_reduce(L, dtype));
}

salt_status salt_reduce_combine(int32_t mode, const double *partials, int64_t count, void *result, salt_dtype dtype,
                                void *hip_stream) {
    if (mode < kModeDot || mode > kModeAsum) return fail(SALT_ERR_ARG, "mode " + std::to_string(mode) + " outside 0..2");
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    if (count < 0) return fail(SALT_ERR_ARG, "negative partial count");
    if (!result) return fail(SALT_ERR_ARG, "result pointer is NULL");
    if (count > 0 && !partials) return fail(SALT_ERR_ARG, "partials pointer is NULL");
    if (((uintptr_t)partials & 7u) != 0) return fail(SALT_ERR_ARG, "partials not 8-byte aligned");
    ReduceLaunch L;
    std::memset(&L, 0, sizeof L);
    L.result = result;
    L.ws = const_cast<double *>(partials);
    L.mode = mode;
    L.passes = 2;
    L.n_partials = count;
    L.stream = hip_stream;
    return device_status(launch_reduce(L, dtype));
}

salt_status salt_scal(int64_t n, double alpha, void *x, int64_t incx, salt_dtype dtype, void *hip_stream) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    if (n == 0 || incx <= 0) return SALT_OK;  // reference BLAS: nothing to do
    salt_status s = check_vec(n, x, incx, "x", true);
    if (s != SALT_OK) return s;
    if (incx == 1) {
        static const uint32_t prog[3] = {SALT_TOKEN(SALT_OP_SCALAR, 0), SALT_TOKEN(SALT_OP_LOAD, 0),
                                         SALT_TOKEN(SALT_OP_MUL, 0)};
        const void *ops[1] = {x};
        return eval_impl(prog, 3, ops, 1, &alpha, 1, x, n, dtype, hip_stream, nullptr);
    }
    StridedMapLaunch L{x, incx, x, incx, n, alpha, kMapScal, hip_stream};
    return device_status(launch_strided_map(L, dtype));
}

salt_status salt_copy(int64_t n, const void *x, int64_t incx, void *y, int64_t incy, salt_dtype dtype,
                      void *hip_stream) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    salt_status s = check_vec(n, x, incx, "x", false);
    if (s == SALT_OK) s = check_vec(n, y, incy, "y", true);
    if (s != SALT_OK || n == 0) return s;
    if (incx == 1 && incy == 1) {
        static const uint32_t prog[1] = {SALT_TOKEN(SALT_OP_LOAD, 0)};
        const void *ops[1] = {x};
        return eval_impl(prog, 1, ops, 1, nullptr, 0, y, n, dtype, hip_stream, nullptr);
    }
    StridedMapLaunch L{x, incx, y, incy, n, 0.0, kMapCopy, hip_stream};
    return device_status(launch_strided_map(L, dtype));
}

salt_status salt_axpy_strided(int64_t n, double alpha, const void *x, int64_t incx, void *y, int64_t incy,
                              salt_dtype dtype, void *hip_stream) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    salt_status s = check_vec(n, x, incx, "x", false);
    if (s == SALT_OK) s = check_vec(n, y, incy, "y", true);
    if (s != SALT_OK || n == 0) return s;
    if (incx == 1 && incy == 1) return salt_axpy(n, alpha, x, y, dtype, hip_stream);
    StridedMapLaunch L{x, incx, y, incy, n, alpha, kMapAxpy, hip_stream};
    return device_status(launch_strided_map(L, dtype));
}

salt_status salt_dot_strided(int64_t n, const void *x, int64_t incx, const void *y, int64_t incy, void *result,
                             void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream) {
    return strided_reduce_impl(n, x, incx, y, incy, result, workspace, ws_bytes, dtype, hip_stream, kModeDot);
}

salt_status salt_nrm2_strided(int64_t n, const void *x, int64_t incx, void *result, void *workspace,
                              size_t ws_bytes, salt_dtype dtype, void *hip_stream) {
    return strided_reduce_impl(n, x, incx, x, incx, result, workspace, ws_bytes, dtype, hip_stream, kModeNrm2);
}

salt_status salt_asum(int64_t n, const void *x, int64_t incx, void *result, void *workspace, size_t ws_bytes,
                      salt_dtype dtype, void *hip_stream) {
    return strided_reduce_impl(n, x, incx, x, incx, result, workspace, ws_bytes, dtype, hip_stream, kModeAsum);
}

salt_status salt_iamax(int64_t n, const void *x, int64_t incx, int64_t *result, void *workspace,
                       size_t ws_bytes, salt_dtype dtype, void *hip_stream) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string(dtype));
    if (n < 0) return fail(SALT_ERR_ARG, "negative length");
    if (!result) return fail(SALT_ERR_ARG, "result pointer is NULL");
    if (incx <= 0) n = 0;  // the answer is -1
    salt_status s = check_vec(n, x, incx, "x", false);
    if (s == SALT_OK)
        s = check_reduce_ws(n, dtype, workspace, ws_bytes, x, span_bytes(n, incx, dtype), nullptr, 0);
    if (s != SALT_OK) return s;
    if (((uintptr_t)result & 7u) != 0) return fail(SALT_ERR_ARG, "result not 8-byte aligned");
    IamaxLaunch L{x, incx, result, (int64_t *)workspace, n, incx == 1 && aligned16(x) ? 1 : 0, hip_stream};
    return device_status(launch_iamax(L, dtype));
}

salt_status salt_nrm2(int64_t n, const void *x, void *result, void *workspace, size_t ws_bytes,
                      salt_dtype dtype, void *hip_stream) {
    return reduce_impl(n, x, x, result, workspace, ws_bytes, dtype, hip_stream, nullptr, kModeNrm2);
}

salt_status salt_nrm2_ex(int64_t n, const void *x, void *result, void *workspace, size_t ws_bytes,
                         salt_dtype dtype, void *hip_stream, const salt_launch_config *cfg) {
    return reduce_impl(n, x, x, result, workspace, ws_bytes, dtype, hip_stream, cfg, kModeNrm2);
}

salt_status salt_dot_expr(const uint32_t *prog_x, int32_t len_x, const uint32_t *prog_y, int32_t len_y,
                          const void *const *operands, int32_t n_operands, const double *scalars,
                          int32_t n_scalars, int64_t n, void *result, void *workspace, size_t ws_bytes,
                          salt_dtype dtype, void *hip_stream) {
    return reduce_expr_impl(prog_x, len_x, prog_y, len_y, operands, n_operands, scalars, n_scalars, n, result,
                            workspace, ws_bytes, dtype, hip_stream, false, nullptr);
}

salt_status salt_dot_expr_ex(const uint32_t *prog_x, int32_t len_x, const uint32_t *prog_y, int32_t len_y,
                             const void *const *operands, int32_t n_operands, const double *scalars,
                             int32_t n_scalars, int64_t n, void *result, void *workspace, size_t ws_bytes,
                             salt_dtype dtype, void *hip_stream, const salt_launch_config *cfg) {
    return reduce_expr_impl(prog_x, len_x, prog_y, len_y, operands, n_operands, scalars, n_scalars, n, result,
                            workspace, ws_bytes, dtype, hip_stream, false, cfg);
}

salt_status salt_nrm2_expr(const uint32_t *prog, int32_t prog_len, const void *const *operands,
                           int32_t n_operands, const double *scalars, int32_t n_scalars, int64_t n, void *result,
                           void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream) {
    return reduce_expr_impl(prog, prog_len, nullptr, 0, operands, n_operands, scalars, n_scalars, n, result,
                            workspace, ws_bytes, dtype, hip_stream, true, nullptr);
}

salt_status salt_nrm2_expr_ex(const uint32_t *prog, int32_t prog_len, const void *const *operands,
                              int32_t n_operands, const double *scalars, int32_t n_scalars, int64_t n,
                              void *result, void *workspace, size_t ws_bytes, salt_dtype dtype, void *hip_stream,
                              const salt_launch_config *cfg) {
    return reduce_expr_impl(prog, prog_len, nullptr, 0, operands, n_operands, scalars, n_scalars, n, result,
                            workspace, ws_bytes, dtype, hip_stream, true, cfg);
}

salt_status salt_stream_reference(int32_t reads, int32_t writes, const void *const *inputs, void *output,
                                  int64_t bytes, void *hip_stream) {
    std::string why;
    const salt_status s = stream_reference_impl(reads, writes, inputs, output, bytes, hip_stream, &why);
    if (s != SALT_OK) return fail(s, why);
    return SALT_OK;
}

salt_status salt_serve_trace(const salt_server_config *cfg, const salt_request *requests, int32_t count,
                             salt_request_result *results) {
    std::string why;
    const salt_status s = serve_trace_impl(cfg, requests, count, results, &why);
    if (s != SALT_OK) return fail(s, why);
    return SALT_OK;
}

salt_status salt_batch_plan_create(const uint32_t *prog, int32_t prog_len, int32_t n_operands,
                                   int32_t n_scalars, const salt_batch_item *items, int32_t count,
                                   salt_dtype dtype, salt_batch_plan *plan) {
    if (!plan) return fail(SALT_ERR_ARG, "plan pointer is NULL");
    *plan = nullptr;
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    if (count < 0) return fail(SALT_ERR_ARG, "negative item count");
    if (count > 0 && !items) return fail(SALT_ERR_ARG, "item array is NULL");
    Program p;
    std::string why;
    salt_status s = compile_program(prog, prog_len, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, why);
    int route = route_of(p);
    if (route == kRouteGeneric) {
        // a tree outside the catalogue: its batched kernels are compiled
        // below, once the items tell whether any wants its dot
        if (jit_mode() == kJitOff)
            return fail(SALT_ERR_UNSUPPORTED,
                        "batched launches of a tree outside the catalogue need run-time compilation, which is off");
        route = kRouteJit;
    }
    const int64_t T = reduce_tile_elems(dtype);
    auto *pl = new (std::nothrow) salt_batch_plan_s;
    if (!pl) return fail(SALT_ERR_ARG, "out of host memory");
    pl->route = route;
    pl->prog = p;
    pl->dtype = dtype;
    pl->count = count;
    const size_t es = esize(dtype);
    int64_t tiles = 0;
    try {
        pl->items.resize(count);
        for (int i = 0; i < count; ++i) {
            const salt_batch_item &it = items[i];
            const std::string at = "item " + std::to_string(i) + ": ";
            if (it.n < 0 || (uint64_t)it.n > (uint64_t)INT64_MAX / 16) {
                delete pl;
                return fail(SALT_ERR_ARG, at + "bad length");
            }
            DevItem d;
            std::memset(&d, 0, sizeof d);
            d.n = it.n;
            d.tile_begin = tiles;
            bool vec = !it.out || aligned16(it.out);
            const size_t bytes = (size_t)it.n * es;
            for (int k = 0; k < p.n_loads; ++k) {
                const void *a = it.operands[p.op_map[k]];
                if (it.n > 0 && !a) {
                    delete pl;
                    return fail(SALT_ERR_ARG, at + "operand " + std::to_string(p.op_map[k]) + " is NULL");
                }
                if (it.out && it.n > 0 && partial_overlap(a, it.out, bytes)) {
                    delete pl;
                    return fail(SALT_ERR_ARG, at + "output partially overlaps an operand");
                }
                d.ops[k] = a;
                vec = vec && aligned16(a);
            }
            for (int j = 0; j < p.n_scal; ++j) {
                d.sc64[j] = it.scalars[p.sc_map[j]];
                d.sc32[j] = (float)it.scalars[p.sc_map[j]];
            }
            d.vec = vec ? 1 : 0;
            d.tree = pl->route;
            d.out = it.n > 0 ? it.out : nullptr;
            d.dot_out = it.dot_out;
            if (it.dot_out) {
                if (p.n_loads < 2 || p.op_map[0] != 0 || p.op_map[1] != 1) {
                    delete pl;
                    return fail(SALT_ERR_UNSUPPORTED,
                                at + "dot needs a program whose first two operands read are operands 0 and 1");
                }
                pl->any_dot = true;
            }
            const int64_t nt = (it.n + T - 1) / T;
            if (tiles + nt > (int64_t)INT32_MAX) {
                delete pl;
                return fail(SALT_ERR_UNSUPPORTED, "too many tiles in one batch");
            }
            for (int64_t t = 0; t < nt; ++t) pl->tiles.push_back(TileRef{i, (int32_t)t});
            tiles += nt;
            pl->total_elems += it.n;
            pl->items[i] = d;
        }
    } catch (...) {
        delete pl;
        return fail(SALT_ERR_ARG, "out of host memory");
    }
    pl->total_tiles = tiles;
    if (route == kRouteJit) {
        s = jit_compile_batch(p, dtype, pl->any_dot, &why);
        if (s != SALT_OK) {
            delete pl;
            return fail(s, why);
        }
    }
    order_tiles(pl->tiles.data(), tiles, pl->items.data(), T);
    pl->table_bytes = round_up(sizeof(DevItem) * (size_t)count + sizeof(TileRef) * (size_t)tiles, 256);
    pl->ws_bytes = pl->any_dot ? sizeof(double) * (size_t)tiles : 0;
    *plan = pl;
    return SALT_OK;
}

salt_status salt_batch_plan_info(salt_batch_plan plan, size_t *table_bytes, size_t *ws_bytes, int64_t *tiles) {
    if (!plan) return fail(SALT_ERR_ARG, "plan is NULL");
    if (table_bytes) *table_bytes = plan->table_bytes;
    if (ws_bytes) *ws_bytes = plan->ws_bytes;
    if (tiles) *tiles = plan->total_tiles;
    return SALT_OK;
}

salt_status salt_batch_upload(salt_batch_plan plan, void *table, size_t table_bytes, void *hip_stream) {
    if (!plan) return fail(SALT_ERR_ARG, "plan is NULL");
    if (!table) return fail(SALT_ERR_ARG, "table pointer is NULL");
    if (((uintptr_t)table & 255u) != 0) return fail(SALT_ERR_ARG, "table not 256-byte aligned");
    if (table_bytes < plan->table_bytes) return fail(SALT_ERR_ARG, "table buffer too small");
    std::vector<char> host(plan->table_bytes, 0);
    std::memcpy(host.data(), plan->items.data(), sizeof(DevItem) * plan->items.size());
    std::memcpy(host.data() + sizeof(DevItem) * plan->items.size(), plan->tiles.data(),
                sizeof(TileRef) * plan->tiles.size());
    if (plan->table_bytes > 0) {
        hipError_t e = hipMemcpyAsync(table, host.data(), plan->table_bytes, hipMemcpyHostToDevice,
                                      (hipStream_t)hip_stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
        if (e != hipSuccess) return device_status(e);
    }
    plan->table = table;
    return SALT_OK;
}

salt_status salt_batch_launch(salt_batch_plan plan, void *workspace, size_t ws_bytes, void *hip_stream,
                              const salt_launch_config *cfg) {
    return batch_launch_impl(plan, workspace, ws_bytes, hip_stream, cfg);
}

salt_status salt_batch_graph_create(salt_batch_plan plan, void *workspace, size_t ws_bytes,
                                    const salt_launch_config *cfg, salt_graph *graph) {
    if (!graph) return fail(SALT_ERR_ARG, "graph pointer is NULL");
    *graph = nullptr;
    // a compiled tree's module is loaded before the capture (loading is not
    // recorded in a graph)
    if (plan && plan->route == kRouteJit) {
        const hipError_t le = jit_batch_load(plan->prog, plan->dtype, plan->any_dot);
        if (le != hipSuccess) return device_status(le);
    }
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return device_status(e);
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return device_status(e);
    }
    const salt_status st = batch_launch_impl(plan, workspace, ws_bytes, s, cfg);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    (void)hipStreamDestroy(s);
    if (st != SALT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return device_status(e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return device_status(e);
    auto *gr = new (std::nothrow) salt_graph_s;
    if (!gr) {
        (void)hipGraphExecDestroy(exec);
        return fail(SALT_ERR_ARG, "out of host memory");
    }
    gr->exec = exec;
    *graph = gr;
    return SALT_OK;
}

salt_status salt_graph_launch(salt_graph graph, void *hip_stream) {
    if (!graph || !graph->exec) return fail(SALT_ERR_ARG, "graph is NULL");
    return device_status(hipGraphLaunch(graph->exec, (hipStream_t)hip_stream));
}

void salt_graph_destroy(salt_graph graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    delete graph;
}

void salt_batch_plan_destroy(salt_batch_plan plan) { delete plan; }

salt_status salt_tuning_load(const char *path) {
    std::vector<TuneRow> rows;
    std::string why;
    const std::string p = path ? std::string(path) : default_tune_path();
    if (!parse_tune(p, rows, &why)) return fail(SALT_ERR_ARG, why);
    auto ix = index_tune(rows);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune = std::move(ix);
    g_tune_loaded = true;
    return SALT_OK;
}

salt_status salt_tuning_lookup(int32_t kind, int32_t route, salt_dtype dtype, int64_t n,
                               salt_launch_config *out) {
    if (!out || kind < 0 || kind > 3 || !dtype_ok(dtype)) return fail(SALT_ERR_ARG, "bad lookup arguments");
    *out = lookup(kind, route, dtype, n, kind == kNrm2 ? 1 : kind == kBatch ? 4 : 2);
    return SALT_OK;
}

int32_t salt_catalogue_count(void) { return (int32_t)catalogue().size(); }

int32_t salt_catalogue_program(int32_t i, uint32_t *tokens, int32_t cap, const char **name) {
    const auto &c = catalogue();
    if (i < 0 || i >= (int32_t)c.size()) return -1;
    if (tokens)
        for (int t = 0; t < c[i].len && t < cap; ++t) tokens[t] = c[i].tok[t];
    if (name) *name = c[i].name;
    return c[i].len;
}

salt_status salt_program_route(const uint32_t *prog, int32_t prog_len, int32_t n_operands,
                               int32_t n_scalars, int32_t *route) {
    Program p;
    std::string why;
    const salt_status s = compile_program(prog, prog_len, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, why);
    if (route) *route = route_of(p);
    return SALT_OK;
}

salt_status salt_reduce_expr_route(const uint32_t *prog_x, int32_t len_x, const uint32_t *prog_y, int32_t len_y,
                                   int32_t n_operands, int32_t n_scalars, salt_dtype dtype, int32_t *route) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    const salt_status s = check_pair(prog_x, len_x, prog_y, len_y, n_operands, n_scalars);
    if (s != SALT_OK) return s;
    int32_t om[SALT_MAX_OPERANDS], sm[SALT_MAX_SCALARS];
    int r = route_pair(prog_x, len_x, prog_y, prog_y ? len_y : 0, om, sm, nullptr);
    if (r < 0 && jit_mode() != kJitOff &&
        jit_pair_ready(pair_trees(prog_x, len_x, prog_y, prog_y ? len_y : 0, om, sm, nullptr), dtype))
        r = SALT_ROUTE_COMPILED;
    if (route) *route = r;
    return SALT_OK;
}

salt_status salt_jit_compile_reduce(const uint32_t *prog_x, int32_t len_x, const uint32_t *prog_y, int32_t len_y,
                                    int32_t n_operands, int32_t n_scalars, salt_dtype dtype) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    salt_status s = check_pair(prog_x, len_x, prog_y, len_y, n_operands, n_scalars);
    if (s != SALT_OK) return s;
    int32_t om[SALT_MAX_OPERANDS], sm[SALT_MAX_SCALARS];
    if (route_pair(prog_x, len_x, prog_y, prog_y ? len_y : 0, om, sm, nullptr) >= 0)
        return SALT_OK;  // a pair with an ahead-of-time kernel
    std::string why;
    s = jit_compile_pair(pair_trees(prog_x, len_x, prog_y, prog_y ? len_y : 0, om, sm, nullptr), dtype, &why);
    if (s != SALT_OK) return fail(s, why);
    return SALT_OK;
}

salt_status salt_jit_code_reduce(const uint32_t *prog_x, int32_t len_x, const uint32_t *prog_y, int32_t len_y,
                                 int32_t n_operands, int32_t n_scalars, salt_dtype dtype, void *buf, size_t cap,
                                 size_t *size) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    if (!size) return fail(SALT_ERR_ARG, "size pointer is NULL");
    const salt_status s = check_pair(prog_x, len_x, prog_y, len_y, n_operands, n_scalars);
    if (s != SALT_OK) return s;
    int32_t om[SALT_MAX_OPERANDS], sm[SALT_MAX_SCALARS];
    const std::vector<char> code =
        jit_pair_code(pair_trees(prog_x, len_x, prog_y, prog_y ? len_y : 0, om, sm, nullptr), dtype);
    *size = code.size();
    if (buf && cap >= code.size() && !code.empty()) std::memcpy(buf, code.data(), code.size());
    return SALT_OK;
}

salt_status salt_jit_set_mode(int32_t mode) {
    if (mode < kJitOff || mode > kJitAuto) return fail(SALT_ERR_ARG, "mode outside 0..2");
    jit_set_mode(mode);
    return SALT_OK;
}

salt_status salt_jit_compile(const uint32_t *prog, int32_t prog_len, int32_t n_operands, int32_t n_scalars,
                             salt_dtype dtype) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    Program p;
    std::string why;
    salt_status s = compile_program(prog, prog_len, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, why);
    if (route_of(p) != kRouteGeneric) return SALT_OK;  // a catalogue tree is compiled already
    s = jit_compile(p, dtype, &why);
    if (s != SALT_OK) return fail(s, why);
    return SALT_OK;
}

salt_status salt_jit_code(const uint32_t *prog, int32_t prog_len, int32_t n_operands, int32_t n_scalars,
                          salt_dtype dtype, void *buf, size_t cap, size_t *size) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    if (!size) return fail(SALT_ERR_ARG, "size pointer is NULL");
    Program p;
    std::string why;
    const salt_status s = compile_program(prog, prog_len, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, why);
    const std::vector<char> code = jit_code(p, dtype);
    *size = code.size();
    if (buf && cap >= code.size() && !code.empty()) std::memcpy(buf, code.data(), code.size());
    return SALT_OK;
}

salt_status salt_eval_route(const uint32_t *prog, int32_t prog_len, int32_t n_operands, int32_t n_scalars,
                            salt_dtype dtype, int32_t *route) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    Program p;
    std::string why;
    const salt_status s = compile_program(prog, prog_len, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, why);
    int r = route_of(p);
    if (r == kRouteGeneric && jit_mode() != kJitOff && jit_ready(p, dtype)) r = SALT_ROUTE_COMPILED;
    if (route) *route = r;
    return SALT_OK;
}

salt_status salt_eval_chunking(int32_t n_loads, int64_t n, salt_dtype dtype, int64_t *chunk_elems,
                               int64_t *launches) {
    if (!dtype_ok(dtype)) return fail(SALT_ERR_ARG, "unknown dtype " + std::to_string((int)dtype));
    if (n < 0 || n_loads < 0 || n_loads > SALT_MAX_OPERANDS) return fail(SALT_ERR_ARG, "bad length or operand count");
    const int64_t c = eval_chunk_elems(n_loads, n, dtype);
    if (chunk_elems) *chunk_elems = c;
    if (launches) *launches = n == 0 ? 0 : (c < n ? n / c : 1);
    return SALT_OK;
}

salt_status salt_program_check(const uint32_t *prog, int32_t prog_len, int32_t n_operands,
                               int32_t n_scalars, int32_t *stack_need, int32_t *n_loads) {
    Program p;
    std::string why;
    const salt_status s = compile_program(prog, prog_len, n_operands, n_scalars, &p, &why);
    if (s != SALT_OK) return fail(s, why);
    if (stack_need) *stack_need = p.stack_need;
    if (n_loads) *n_loads = p.n_loads;
    return SALT_OK;
}

const char *salt_status_string(salt_status s) {
    switch (s) {
        case SALT_OK: return "ok";
        case SALT_ERR_ARG: return "invalid argument";
        case SALT_ERR_PROGRAM: return "invalid program";
        case SALT_ERR_UNSUPPORTED: return "unsupported";
        case SALT_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case SALT_ERR_DEVICE: return "device error";
        default: return "unknown status";
    }
}

const char *salt_last_error(void) { return t_err.c_str(); }

int32_t salt_version(void) { return 10000; }

}  // extern "C"
