// jit.hip -- run-time compilation of trees outside the catalogue (jit.hpp).
#include "jit.hpp"

#include <hip/hiprtc.h>

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>

#include "batch.hpp"
#include "reduce_tree.hpp"
#include "salt.h"

namespace salt {
namespace {

// ---- source generation -----------------------------------------------------

// Element-type helpers of the generated code: the same conversions as the
// library's own kernels (device.hpp), so results are bit-identical.
const char *type_block(int dtype) {
    switch (dtype) {
        case SALT_F64:
            return R"(typedef double C;
typedef double f64x2 __attribute__((ext_vector_type(2)));
constexpr int V = 2;
__device__ __forceinline__ C get(const u32x4 &c, int p) { return __builtin_bit_cast(f64x2, c)[p]; }
__device__ __forceinline__ u32x4 pack(const C *v) { f64x2 r; r[0] = v[0]; r[1] = v[1]; return __builtin_bit_cast(u32x4, r); }
__device__ __forceinline__ C ld1(const void *p, long long i) { return ((const double *)p)[i]; }
__device__ __forceinline__ void st1(void *p, long long i, C v) { ((double *)p)[i] = v; }
)";
        case SALT_F32:
            return R"(typedef float C;
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int V = 4;
__device__ __forceinline__ C get(const u32x4 &c, int p) { return __builtin_bit_cast(f32x4, c)[p]; }
__device__ __forceinline__ u32x4 pack(const C *v) { f32x4 r; r[0] = v[0]; r[1] = v[1]; r[2] = v[2]; r[3] = v[3]; return __builtin_bit_cast(u32x4, r); }
__device__ __forceinline__ C ld1(const void *p, long long i) { return ((const float *)p)[i]; }
__device__ __forceinline__ void st1(void *p, long long i, C v) { ((float *)p)[i] = v; }
)";
        case SALT_BF16:
            return R"(typedef float C;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
constexpr int V = 8;
__device__ __forceinline__ C get(const u32x4 &c, int p) {
    const unsigned w = c[p >> 1];
    return __builtin_bit_cast(float, (p & 1) ? (w & 0xffff0000u) : (w << 16));
}
__device__ __forceinline__ unsigned pack2(C lo, C hi) {
    f32x2 f; f[0] = lo; f[1] = hi;
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2));
}
__device__ __forceinline__ u32x4 pack(const C *v) {
    u32x4 r; r[0] = pack2(v[0], v[1]); r[1] = pack2(v[2], v[3]); r[2] = pack2(v[4], v[5]); r[3] = pack2(v[6], v[7]);
    return r;
}
__device__ __forceinline__ C ld1(const void *p, long long i) {
    return __builtin_bit_cast(float, (unsigned)((const unsigned short *)p)[i] << 16);
}
__device__ __forceinline__ void st1(void *p, long long i, C v) {
    ((unsigned short *)p)[i] = __builtin_bit_cast(unsigned short, (__bf16)v);
}
)";
        default:  // the narrowing goes through an opaque value, as in device.hpp
            return R"(typedef float C;
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
constexpr int V = 8;
__device__ __forceinline__ float opaque_f32(float v) { asm("" : "+v"(v)); return v; }
__device__ __forceinline__ C get(const u32x4 &c, int p) { return (float)__builtin_bit_cast(f16x8, c)[p]; }
__device__ __forceinline__ u32x4 pack(const C *v) {
    f16x8 r;
    for (int p = 0; p < 8; ++p) r[p] = (_Float16)opaque_f32(v[p]);
    return __builtin_bit_cast(u32x4, r);
}
__device__ __forceinline__ C ld1(const void *p, long long i) { return (float)((const _Float16 *)p)[i]; }
__device__ __forceinline__ void st1(void *p, long long i, C v) { ((_Float16 *)p)[i] = (_Float16)opaque_f32(v); }
)";
    }
}

// The tree as one C++ expression over x0..x(NL-1) and s[0..], every
// operation parenthesised (one IEEE operation each, postfix order).
std::string infix(const Program &p) {
    std::vector<std::string> st;
    for (int t = 0; t < p.len; ++t) {
        const uint32_t op = p.canon[t] & 0xffu, arg = p.canon[t] >> 8;
        if (op == SALT_OP_LOAD) {
            st.push_back("x" + std::to_string(arg));
        } else if (op == SALT_OP_SCALAR) {
            st.push_back("s[" + std::to_string(arg) + "]");
        } else {
            const std::string r = st.back();
            st.pop_back();
            const std::string l = st.back();
            st.pop_back();
            const char *o = op == SALT_OP_ADD ? " + " : op == SALT_OP_SUB ? " - " : " * ";
            st.push_back("(" + l + o + r + ")");
        }
    }
    return st.empty() ? "(C)0" : st.back();
}

// Chunks per lane of each compiled variant, and the names of the entries.
constexpr int kUnrolls[3] = {1, 2, 4};
std::string entry_name(int u, bool nt) { return "salt_jit_u" + std::to_string(u) + (nt ? "_nt" : "_c"); }

// Host-side image of the generated kernel's argument (the two layouts).
template <class C>
struct JitArgs {
    const void *ops[SALT_MAX_OPERANDS];
    C sc[SALT_MAX_SCALARS];
    void *out;
    long long n;
    int vec;
};

}  // namespace

std::string jit_source(const Program &p, int dtype) {
    const int nl = p.n_loads;
    std::string s;
    s += "// generated by libsalt for one expression tree\n#pragma clang fp contract(off)\n";
    s += "typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));\n";
    s += type_block(dtype);
    s += R"(template <bool NT> __device__ __forceinline__ u32x4 ld16(const u32x4 *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p); else return *p;
}
template <bool NT> __device__ __forceinline__ void st16(u32x4 *p, u32x4 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
}
struct A { const void *ops[8]; C sc[8]; void *out; long long n; int vec; };
)";
    // the tree
    s += "__device__ __forceinline__ C ev(";
    for (int k = 0; k < nl; ++k) s += "C x" + std::to_string(k) + ", ";
    s += "const C *s) { (void)s; return " + infix(p) + "; }\n";
    const int NL = nl > 0 ? nl : 1;
    s += "constexpr int NL = " + std::to_string(NL) + ";\n";
    // the loop: tiles of 256 x U chunks, loads first, then the tree, then the
    // stores; elements after the last whole tile (and all of them when an
    // array is not 16-byte aligned) one by one
    s += R"(template <int U, bool NT> __device__ __forceinline__ void body(const A &a) {
    constexpr long long tile = 256LL * U * V;
    const long long n_tiles = a.vec ? a.n / tile : 0;
    for (long long t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const long long c0 = t * (256LL * U) + threadIdx.x;
        u32x4 raw[NL][U];
)";
    if (nl > 0)
        s += R"(#pragma unroll
        for (int k = 0; k < NL; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) raw[k][u] = ld16<NT>((const u32x4 *)a.ops[k] + c0 + u * 256);
)";
    s += R"(        u32x4 res[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            C r[V];
#pragma unroll
            for (int p = 0; p < V; ++p) r[p] = ev()";
    for (int k = 0; k < nl; ++k) s += "get(raw[" + std::to_string(k) + "][u], p), ";
    s += R"(a.sc);
            res[u] = pack(r);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) st16<NT>((u32x4 *)a.out + c0 + u * 256, res[u]);
    }
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = n_tiles * tile + (long long)blockIdx.x * 256 + threadIdx.x; i < a.n; i += stride)
        st1(a.out, i, ev()";
    for (int k = 0; k < nl; ++k) s += "ld1(a.ops[" + std::to_string(k) + "], i), ";
    s += "a.sc));\n}\n";
    for (int u : kUnrolls)
        for (int nt = 0; nt < 2; ++nt)
            s += "extern \"C\" __global__ __launch_bounds__(256) void " + entry_name(u, nt) + "(A a) { body<" +
                 std::to_string(u) + ", " + (nt ? "true" : "false") + ">(a); }\n";
    return s;
}

// ---- reduction pairs ---------------------------------------------------------

namespace {

// The tree as a type of expr.hpp (Ld / Sc / Bin), from canonical postfix.
std::string tree_type(const uint32_t *tok, int len) {
    std::vector<std::string> st;
    for (int t = 0; t < len; ++t) {
        const uint32_t op = tok[t] & 0xffu, arg = tok[t] >> 8;
        if (op == SALT_OP_LOAD) {
            st.push_back("Ld<" + std::to_string(arg) + ">");
        } else if (op == SALT_OP_SCALAR) {
            st.push_back("Sc<" + std::to_string(arg) + ">");
        } else {
            const std::string r = st.back();
            st.pop_back();
            const std::string l = st.back();
            st.pop_back();
            st.push_back("Bin<" + std::to_string(op) + ", " + l + ", " + r + ">");
        }
    }
    return st.empty() ? "NoTree" : st.back();
}

// Chunks per lane of the compiled pass-1 variants.
constexpr int kPairUnrolls[3] = {2, 4, 8};

std::string pair_kernel_expr(int dtype, int u, bool nt) {
    return "salt::k_reduce_tree<salt::jit_pair::P, salt::jit_pair::Q, " + std::to_string(dtype) + ", " +
           std::to_string(u) + ", " + (nt ? "true" : "false") + ">";
}

}  // namespace

std::string jit_pair_source(const PairTrees &t, int dtype) {
    (void)dtype;  // the element type is a template argument of the kernels
    std::string s;
    s += "// generated by libsalt for one reduction pair\n#include \"reduce_tree.hpp\"\n";
    s += "namespace salt {\nnamespace jit_pair {\n";
    s += "using P = " + tree_type(t.p, t.lp) + ";\n";
    s += "using Q = " + (t.nrm2 ? std::string("NoTree") : tree_type(t.q, t.lq)) + ";\n";
    s += "}  // namespace jit_pair\n}  // namespace salt\n";
    return s;
}

std::string jit_batch_source(const Program &p, int dtype) {
    (void)dtype;  // the element type is a template argument of the kernels
    std::string s;
    s += "// generated by libsalt for one tree in batched launches\n#include \"batch_device.hpp\"\n";
    s += "namespace salt {\nnamespace jit_batch {\n";
    s += "using E = " + tree_type(p.canon, p.len) + ";\n";
    s += "}  // namespace jit_batch\n}  // namespace salt\n";
    return s;
}

namespace {

std::string batch_kernel_expr(int dtype, int u, bool nt, bool dot) {
    return "salt::k_batch<salt::jit_batch::E, " + std::to_string(dtype) + ", " + std::to_string(u) + ", " +
           (nt ? "true" : "false") + ", " + (dot ? "true" : "false") + ">";
}

// ---- cache and per-device modules -----------------------------------------

enum State { kNew = 0, kCompiling = 1, kCompiled = 2, kFailed = 3 };
enum Kind { kKindEval = 0, kKindPair = 1, kKindBatch = 2 };

// Kernel variants of a module: 3 unroll choices x (cached, streaming) x
// (without, with the batched dot); element-wise trees and reduction pairs
// use the first half only.
constexpr int kVariants = 12;
constexpr int vidx(int ui, bool nt, bool dot) { return (ui * 2 + (nt ? 1 : 0)) * 2 + (dot ? 1 : 0); }

struct Loaded {
    hipModule_t mod = nullptr;
    hipFunction_t fn[kVariants] = {};
};

struct Entry {
    std::atomic<int> state{kNew};
    int seen = 0;  // large calls that found it not compiled (automatic mode)
    int kind = kKindEval;
    Program prog;      // an element-wise tree
    PairTrees pair;    // a reduction pair
    bool dot = false;  // batched: the variants with the fused dot (else without)
    int dtype = 0;
    std::vector<char> code;
    std::string log;
    std::string names[kVariants];  // kernel symbols by vidx (empty: not built)
    std::map<int, Loaded> dev;  // device -> loaded module
};

std::string key_of(const Program &p, int dtype) {
    std::string k(1, (char)('0' + dtype));
    k.append((const char *)p.canon, sizeof(uint32_t) * (size_t)p.len);
    return k;
}

std::string batch_key_of(const Program &p, int dtype, bool dot) {
    std::string k = "b";
    k += (char)('0' + dtype);
    k += dot ? 'd' : 'e';
    k.append((const char *)p.canon, sizeof(uint32_t) * (size_t)p.len);
    return k;
}

std::string key_of(const PairTrees &t, int dtype) {
    std::string k = "r";
    k += (char)('0' + dtype);
    k += t.nrm2 ? 'n' : 'd';
    k += (char)t.lp;
    k.append((const char *)t.p, sizeof(uint32_t) * (size_t)t.lp);
    if (!t.nrm2) k.append((const char *)t.q, sizeof(uint32_t) * (size_t)t.lq);
    return k;
}

// Headers a generated pair kernel includes: the runtime's own headers are
// built into the run-time compiler, so their names resolve to stubs here,
// and the library's headers come from the text embedded at build time.
#include "jit_headers.inc"

const char kStubEmpty[] = "#pragma once\n";
const char kStubStdint[] =
    "#pragma once\n"
    "typedef __INT8_TYPE__ int8_t;\ntypedef __INT16_TYPE__ int16_t;\n"
    "typedef __INT32_TYPE__ int32_t;\ntypedef __INT64_TYPE__ int64_t;\n"
    "typedef __UINT8_TYPE__ uint8_t;\ntypedef __UINT16_TYPE__ uint16_t;\n"
    "typedef __UINT32_TYPE__ uint32_t;\ntypedef __UINT64_TYPE__ uint64_t;\n"
    "typedef __INTPTR_TYPE__ intptr_t;\ntypedef __UINTPTR_TYPE__ uintptr_t;\n";
const char kStubStddef[] = "#pragma once\ntypedef __SIZE_TYPE__ size_t;\ntypedef __PTRDIFF_TYPE__ ptrdiff_t;\n";

bool compile_entry(Entry &e) {
    // reduction pairs and batched trees are built from the embedded headers
    const bool pair = e.kind != kKindEval;
    const std::string src = e.kind == kKindPair    ? jit_pair_source(e.pair, e.dtype)
                            : e.kind == kKindBatch ? jit_batch_source(e.prog, e.dtype)
                                                   : jit_source(e.prog, e.dtype);
    std::vector<const char *> hnames, htexts;
    if (pair) {
        hnames = {"hip/hip_runtime.h", "cstdint", "stdint.h", "stddef.h"};
        htexts = {kStubEmpty, kStubStdint, kStubStdint, kStubStddef};
        for (int i = 0; i < kJitHeaderCount; ++i) {
            hnames.push_back(kJitHeaderNames[i]);
            htexts.push_back(kJitHeaderTexts[i]);
        }
    }
    hiprtcProgram h;
    if (hiprtcCreateProgram(&h, src.c_str(), pair ? "salt_jit_pair.hip" : "salt_jit.hip", (int)hnames.size(),
                            htexts.data(), hnames.data()) != HIPRTC_SUCCESS) {
        e.log = "hiprtcCreateProgram failed";
        return false;
    }
    // the instantiations to build, by variant (template kernels are named by
    // expression and looked up by their lowered names after compiling)
    std::string exprs[kVariants];
    if (pair)
        for (int i = 0; i < 3; ++i)
            for (int nt = 0; nt < 2; ++nt)
                for (int dot = 0; dot < 2; ++dot) {
                    std::string &x = exprs[vidx(i, nt != 0, dot != 0)];
                    if (e.kind == kKindPair && !dot)
                        x = pair_kernel_expr(e.dtype, kPairUnrolls[i], nt != 0);
                    else if (e.kind == kKindBatch && (dot != 0) == e.dot)
                        x = batch_kernel_expr(e.dtype, kPairUnrolls[i], nt != 0, dot != 0);
                    if (!x.empty() && hiprtcAddNameExpression(h, x.c_str()) != HIPRTC_SUCCESS) {
                        e.log = "hiprtcAddNameExpression failed";
                        hiprtcDestroyProgram(&h);
                        return false;
                    }
                }
    // the library's own build rules: no contraction, no packed binary32
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(h, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t ls = 0;
    hiprtcGetProgramLogSize(h, &ls);
    if (ls > 1) {
        e.log.assign(ls, '\0');
        hiprtcGetProgramLog(h, &e.log[0]);
    }
    bool ok = r == HIPRTC_SUCCESS;
    if (ok) {
        size_t cs = 0;
        ok = hiprtcGetCodeSize(h, &cs) == HIPRTC_SUCCESS && cs > 0;
        if (ok) {
            e.code.resize(cs);
            ok = hiprtcGetCode(h, e.code.data()) == HIPRTC_SUCCESS;
        }
        for (int i = 0; i < 3 && ok; ++i)
            for (int nt = 0; nt < 2 && ok; ++nt) {
                if (!pair) {
                    e.names[vidx(i, nt != 0, false)] = entry_name(kUnrolls[i], nt != 0);
                    continue;
                }
                for (int dot = 0; dot < 2 && ok; ++dot) {
                    const std::string &x = exprs[vidx(i, nt != 0, dot != 0)];
                    if (x.empty()) continue;
                    const char *lowered = nullptr;
                    ok = hiprtcGetLoweredName(h, x.c_str(), &lowered) == HIPRTC_SUCCESS && lowered;
                    if (ok) e.names[vidx(i, nt != 0, dot != 0)] = lowered;  // copied before the destroy
                    else e.log += "\nno symbol for " + x;
                }
            }
    } else if (e.log.empty()) {
        e.log = hiprtcGetErrorString(r);
    }
    hiprtcDestroyProgram(&h);
    return ok;
}

// Compilation runs on the calling thread. (A library thread compiling in
// the background could still be inside the compiler when the process
// exits; the compiler library, loaded at the first compile, would then be
// torn down under it.) Entries are never freed: they live until the
// process ends.
struct Jit {
    std::mutex mu;
    std::map<std::string, Entry *> cache;
    std::atomic<int> mode{kJitAuto};
};

Jit &jit() {
    static Jit *j = new Jit;
    return *j;
}

// The entry of `key`, created by init if absent (with mu held).
template <class Init>
Entry *entry_locked(Jit &J, const std::string &key, const Init &init) {
    Entry *&slot = J.cache[key];
    if (!slot) {
        slot = new Entry;
        init(*slot);
    }
    return slot;
}

Entry *find_locked(Jit &J, const std::string &key) {
    auto it = J.cache.find(key);
    return it == J.cache.end() ? nullptr : it->second;
}

// Compile an entry this thread has claimed (state kCompiling), without mu.
void compile_claimed(Entry *e) {
    const bool ok = compile_entry(*e);
    e->state.store(ok ? kCompiled : kFailed);
}

// The loaded module of a compiled entry on the current device (with mu held).
hipError_t loaded_locked(Entry &e, Loaded **out) {
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    auto it = e.dev.find(dev);
    if (it == e.dev.end()) {
        Loaded l;
        err = hipModuleLoadData(&l.mod, e.code.data());
        if (err != hipSuccess) return err;
        for (int v = 0; v < kVariants; ++v) {
            if (e.names[v].empty()) continue;
            err = hipModuleGetFunction(&l.fn[v], l.mod, e.names[v].c_str());
            if (err != hipSuccess) {
                (void)hipModuleUnload(l.mod);
                return err;
            }
        }
        it = e.dev.emplace(dev, l).first;
    }
    *out = &it->second;
    return hipSuccess;
}

// The module to launch for `key` on the current device, or null when the
// call should run on the library's own kernels: not compiled yet (in the
// automatic mode a key's second call of at least kJitAutoMinElems elements
// compiles it here first), compiling on another thread, failed, or not
// loaded on this device while the stream is being captured.
template <class Init>
hipError_t acquire(const std::string &key, const Init &init, int64_t n, hipStream_t stream, Loaded **out) {
    *out = nullptr;
    Jit &J = jit();
    const int mode = J.mode.load();
    if (mode == kJitOff) return hipSuccess;
    Entry *claimed = nullptr;
    {
        std::lock_guard<std::mutex> g(J.mu);
        Entry *e = find_locked(J, key);
        if (!e || e->state.load() == kNew) {
            // automatic mode: compiled on its second large call (the first
            // runs on the library's kernels), so one-off trees cost nothing
            if (mode != kJitAuto || n < kJitAutoMinElems) return hipSuccess;
            e = entry_locked(J, key, init);
            if (++e->seen < 2) return hipSuccess;
            e->state.store(kCompiling);
            claimed = e;
        } else if (e->state.load() != kCompiled) {
            return hipSuccess;  // compiling elsewhere, or failed
        }
    }
    if (claimed) {
        compile_claimed(claimed);
        if (claimed->state.load() != kCompiled) return hipSuccess;
    }
    std::lock_guard<std::mutex> g(J.mu);
    Entry *e = find_locked(J, key);
    // loading a module during stream capture is not recorded in the graph;
    // a key not yet loaded on this device runs on the library's kernels there
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();  // leave no error behind for the fallback's launch
        return hipSuccess;
    }
    if (!e->dev.count(dev)) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
            (void)hipGetLastError();
            return hipSuccess;
        }
        if (cs != hipStreamCaptureStatusNone) return hipSuccess;
    }
    return loaded_locked(*e, out);
}

// Compile `key` now on the calling thread (or wait for the thread that is).
template <class Init>
salt_status compile_now(const std::string &key, const Init &init, std::string *err) {
    Jit &J = jit();
    Entry *e = nullptr;
    bool mine = false;
    {
        std::lock_guard<std::mutex> g(J.mu);
        e = entry_locked(J, key, init);
        int expect = kNew;
        mine = e->state.compare_exchange_strong(expect, kCompiling);
    }
    if (mine) compile_claimed(e);
    while (e->state.load() == kCompiling) std::this_thread::yield();  // another thread compiles it
    if (e->state.load() != kCompiled) {
        *err = "compilation failed: " + e->log;
        return SALT_ERR_UNSUPPORTED;
    }
    return SALT_OK;
}

std::vector<char> code_of(const std::string &key) {
    Jit &J = jit();
    std::lock_guard<std::mutex> g(J.mu);
    Entry *e = find_locked(J, key);
    if (!e || e->state.load() != kCompiled) return {};
    return e->code;
}

int ready(const std::string &key) {
    Jit &J = jit();
    std::lock_guard<std::mutex> g(J.mu);
    Entry *e = find_locked(J, key);
    return e && e->state.load() == kCompiled ? 1 : 0;
}

template <class C>
hipError_t launch_jit(const Loaded &l, const EvalLaunch &L, int dtype, int n_loads) {
    JitArgs<C> a;
    std::memset(&a, 0, sizeof a);
    for (int k = 0; k < SALT_MAX_OPERANDS; ++k) a.ops[k] = L.ops[k];
    for (int j = 0; j < SALT_MAX_SCALARS; ++j) a.sc[j] = (C)L.sc[j];  // rounded once to the compute type
    a.out = L.out;
    a.n = L.n;
    a.vec = L.vec;
    // chunks per lane: the launch knob's unroll (8 runs as 4), at most 2
    // with more than four operands (register budget)
    int ui = L.unroll >= 4 ? 2 : L.unroll == 2 ? 1 : 0;
    if (n_loads > 4 && ui > 1) ui = 1;
    const int u = kUnrolls[ui];
    const int V = dtype == SALT_F64 ? 2 : dtype == SALT_F32 ? 4 : 8;
    const int64_t tile = (int64_t)256 * u * V;
    const int64_t n_tiles = L.vec ? L.n / tile : 0;
    int64_t g;
    if (n_tiles > 0) {
        g = L.blocks > 0 ? (L.blocks < n_tiles ? L.blocks : n_tiles) : n_tiles;
    } else {
        g = (L.n + 255) / 256;
        const int64_t cap = L.blocks > 0 ? L.blocks : 8192;
        if (g > cap) g = cap;
    }
    if (g < 1) g = 1;
    if (g > 0x7fffffff) g = 0x7fffffff;
    void *params[] = {&a};
    return hipModuleLaunchKernel(l.fn[vidx(ui, L.nontemporal != 0, false)], (unsigned)g, 1, 1, 256, 1, 1, 0,
                                 (hipStream_t)L.stream, params, nullptr);
}

// Pass 1 of a compiled pair: the argument block is the template's own
// RedTreeArgs, so host and kernel agree on its layout.
template <int DT>
hipError_t launch_pair(const Loaded &l, const ReduceExprLaunch &L, int n_loads) {
    RedTreeArgs<DT> a;
    std::memset(&a, 0, sizeof a);
    for (int k = 0; k < SALT_MAX_OPERANDS; ++k) a.ops[k] = L.ops[k];
    for (int j = 0; j < SALT_MAX_SCALARS; ++j) a.sc[j] = (typename Tr<DT>::C)L.sc[j];
    const int64_t T = tile_elems<DT>();
    const int64_t n_tiles = (L.n + T - 1) / T;
    a.ws = L.ws;
    a.n = L.n;
    a.vec = L.vec;
    a.result = L.result;
    a.final_store = n_tiles == 1 ? 1 : 0;
    // chunks per lane per burst: the knob's unroll (16 runs as 8), lowered
    // with more operands (register budget: operands x chunks <= 16)
    int ui = L.unroll >= 8 ? 2 : L.unroll == 4 ? 1 : 0;
    if (n_loads > 2 && ui > 1) ui = 1;
    if (n_loads > 4) ui = 0;
    int64_t grid = L.blocks > 0 && L.blocks < n_tiles ? L.blocks : n_tiles;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    void *params[] = {&a};
    return hipModuleLaunchKernel(l.fn[vidx(ui, L.nontemporal != 0, false)], (unsigned)grid, 1, 1, kBlock, 1, 1, 0,
                                 (hipStream_t)L.stream, params, nullptr);
}

// The batched kernel of a compiled tree (the template's own argument list),
// then the library's per-item combine when any item wants its dot.
hipError_t launch_batch(const Loaded &l, const BatchLaunch &L, int dtype, int n_loads) {
    // chunks per burst: the knob's unroll, at most 4 with more than four
    // operands (register budget)
    int ui = L.unroll >= 8 ? 2 : L.unroll == 4 ? 1 : 0;
    if (n_loads > 4 && ui > 1) ui = 1;
    const bool dot = L.any_dot != 0;
    hipFunction_t f = l.fn[vidx(ui, L.nontemporal != 0, dot)];
    if (!f) return hipErrorInvalidValue;  // a dot needs two operands (the planner checks it)
    int64_t grid = L.blocks > 0 && L.blocks < L.total_tiles ? L.blocks : L.total_tiles;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    if (grid > 0) {
        const DevItem *items = L.items;
        const TileRef *tiles = L.tiles;
        int64_t total = L.total_tiles;
        double *ws = L.ws;
        void *params[] = {&items, &tiles, &total, &ws};
        const hipError_t e = hipModuleLaunchKernel(f, (unsigned)grid, 1, 1, kBlock, 1, 1, 0,
                                                   (hipStream_t)L.stream, params, nullptr);
        if (e != hipSuccess) return e;
    }
    if (!dot) return hipSuccess;
    BatchFn combine = batch_combine_launcher(dtype);
    return combine ? (hipError_t)combine(L) : hipErrorInvalidValue;
}

// The loaded module of a compiled batched tree on the current device;
// loading is refused while `stream` is being captured (it would not be
// recorded), and an entry that is not compiled is an error: batched plans
// compile their tree when they are created.
hipError_t batch_module(const Program &p, int dtype, bool dot, hipStream_t stream, bool capture_ok,
                        Loaded **out) {
    *out = nullptr;
    Jit &J = jit();
    std::lock_guard<std::mutex> g(J.mu);
    Entry *e = find_locked(J, batch_key_of(p, dtype, dot));
    if (!e || e->state.load() != kCompiled) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (!e->dev.count(dev) && !capture_ok) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        err = hipStreamIsCapturing(stream, &cs);
        if (err != hipSuccess) return err;
        if (cs != hipStreamCaptureStatusNone) return hipErrorStreamCaptureUnsupported;
    }
    return loaded_locked(*e, out);
}

}  // namespace

salt_status jit_compile_batch(const Program &p, int dtype, bool dot, std::string *err) {
    if (dot && p.n_loads < 2) {
        *err = "a dot needs two operands";
        return SALT_ERR_UNSUPPORTED;
    }
    return compile_now(
        batch_key_of(p, dtype, dot),
        [&](Entry &e) {
            e.kind = kKindBatch;
            e.prog = p;
            e.dtype = dtype;
            e.dot = dot;
        },
        err);
}

hipError_t jit_batch_load(const Program &p, int dtype, bool dot) {
    Loaded *l = nullptr;
    return batch_module(p, dtype, dot, nullptr, true, &l);
}

hipError_t jit_batch_launch(const BatchLaunch &L, const Program &p, int dtype) {
    Loaded *l = nullptr;
    const hipError_t err = batch_module(p, dtype, L.any_dot != 0, (hipStream_t)L.stream, false, &l);
    if (err != hipSuccess) return err;
    return launch_batch(*l, L, dtype, p.n_loads);
}

std::vector<char> jit_batch_code(const Program &p, int dtype, bool dot) {
    return code_of(batch_key_of(p, dtype, dot));
}

hipError_t jit_try_launch(const EvalLaunch &L, const Program &p, int dtype, bool *ran) {
    *ran = false;
    Loaded *l = nullptr;
    const hipError_t err = acquire(
        key_of(p, dtype),
        [&](Entry &e) {
            e.kind = kKindEval;
            e.prog = p;
            e.dtype = dtype;
        },
        L.n, (hipStream_t)L.stream, &l);
    if (err != hipSuccess || !l) return err;
    *ran = true;
    if (dtype == SALT_F64) return launch_jit<double>(*l, L, dtype, p.n_loads);
    return launch_jit<float>(*l, L, dtype, p.n_loads);
}

hipError_t jit_try_reduce(const ReduceExprLaunch &L, const PairTrees &t, int dtype, bool *ran) {
    *ran = false;
    if (L.n <= 0) return hipSuccess;  // nothing for pass 1: the library stores the zero
    Loaded *l = nullptr;
    const hipError_t err = acquire(
        key_of(t, dtype),
        [&](Entry &e) {
            e.kind = kKindPair;
            e.pair = t;
            e.dtype = dtype;
        },
        L.n, (hipStream_t)L.stream, &l);
    if (err != hipSuccess || !l) return err;
    *ran = true;
    switch (dtype) {
        case SALT_F64: return launch_pair<SALT_F64>(*l, L, t.n_loads);
        case SALT_F32: return launch_pair<SALT_F32>(*l, L, t.n_loads);
        case SALT_BF16: return launch_pair<SALT_BF16>(*l, L, t.n_loads);
        default: return launch_pair<SALT_F16>(*l, L, t.n_loads);
    }
}

salt_status jit_compile(const Program &p, int dtype, std::string *err) {
    return compile_now(
        key_of(p, dtype),
        [&](Entry &e) {
            e.kind = kKindEval;
            e.prog = p;
            e.dtype = dtype;
        },
        err);
}

salt_status jit_compile_pair(const PairTrees &t, int dtype, std::string *err) {
    return compile_now(
        key_of(t, dtype),
        [&](Entry &e) {
            e.kind = kKindPair;
            e.pair = t;
            e.dtype = dtype;
        },
        err);
}

std::vector<char> jit_code(const Program &p, int dtype) { return code_of(key_of(p, dtype)); }
std::vector<char> jit_pair_code(const PairTrees &t, int dtype) { return code_of(key_of(t, dtype)); }
int jit_ready(const Program &p, int dtype) { return ready(key_of(p, dtype)); }
int jit_pair_ready(const PairTrees &t, int dtype) { return ready(key_of(t, dtype)); }

void jit_set_mode(int mode) { jit().mode.store(mode); }
int jit_mode() { return jit().mode.load(); }

}  // namespace salt
