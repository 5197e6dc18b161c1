/*
 * salt_oracle.c -- plain, slow, obviously correct CPU reference for the SALT
 * hot path (fused element-wise vector expressions, axpy, dot, nrm2).
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only code allowed to load this
 * library. The GPU product path never calls it, and the two share no code.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 *        -fno-fast-math (contraction off: every add, sub and mul is one IEEE
 *        operation).
 *
 * What is computed, and the passage each function follows:
 *  - oracle_eval_*: the expression tree is evaluated lazily at assignment,
 *    once per element, one loop over all elements (Sec. 2, Fig. 1: the tree
 *    for d = a + (b - c); fusion keeps intermediates in registers and does not
 *    change the per-element arithmetic). The tree arrives in postfix form; it
 *    is run as a stack machine per element, each ADD/SUB/MUL rounded once to
 *    the compute precision, round-to-nearest-even, no contraction.
 *  - oracle_axpy_*: y = y + alpha*x (Sec. 5, the xAXPY benchmark), i.e. the
 *    tree [SCALAR0 LOAD0 MUL LOAD1 ADD] written as its plain definition.
 *  - oracle_dot2: the dot product reduction at the root of a tree (Sec. 2,
 *    "dot product or norm"; Sec. 4.2, the reduction step). A reduction's order
 *    is not fixed by the paper, so only the exact real value is well defined;
 *    the oracle approximates it with Dot2 (Ogita, Rump and Oishi, "Accurate
 *    sum and dot product", SIAM J. Sci. Comput. 26(6), 2005, Alg. 5.3), whose
 *    error is at most u|x.y| + gamma_n^2 |x|.|y| in binary64.
 *  - oracle_nrm2: the "norm" of Sec. 2, read as the unscaled 2-norm
 *    sqrt(sum x_i^2), from Dot2(x, x).
 *  - oracle_naive_dot_*: plain sequential loops, kept as a CPU timing baseline
 *    and as the same-precision FP32 mode (not a reference value at large n).
 *    oracle_naive_dot_f64_par is the all-cores form of the binary64 loop:
 *    each of T threads sums one contiguous share of the elements in order,
 *    and the T partial sums are added in thread order (the OpenMP layer of
 *    Sec. 6 applied to the timing baseline).
 *  - oracle_set_threads: the element-wise loops (eval, axpy) run on that many
 *    host threads, OpenMP static shares of the element range. Each element is
 *    computed alone, so the results do not depend on the thread count.
 *  - oracle_reduce_canonical: a second, bit-exact reduction oracle. The
 *    paper's reduction keeps per-slot partial sums and ends with a
 *    reduction step (Sec. 4.2) without fixing an order; the library fixes
 *    one that depends on (n, storage type) only, so its results are
 *    reproducible. This replays that documented order on the CPU, in the
 *    same precisions, so dot, nrm2 and asum can be compared bit for bit
 *    (the order is a reading of the paper, written out below).
 *  - oracle_copy, oracle_iamax_*: the BLAS level-1 interface that the paper
 *    measures against (Sec. 1, the BLAS interface; Sec. 5, the xDOT / xSCAL /
 *    xAXPY / xCOPY comparisons), with its strided vectors. A BLAS vector of n
 *    elements with increment inc holds element i at x[i*inc] for inc >= 0
 *    and at x[(n-1-i)*(-inc)] for inc < 0 (the reference BLAS convention).
 *    Strided scal, axpy, dot, nrm2 and asum are these gathers followed by the
 *    contiguous definitions above (composed in oracle/__init__.py).
 *
 * Storage types: binary64 ("f64"), binary32 ("f32"), bfloat16 and binary16
 * held as raw 16-bit patterns. 16-bit storage is widened exactly to binary32,
 * computed in binary32, and narrowed once with round-to-nearest-even; the
 * widening and narrowing below are written from the formats' definitions.
 *
 * Program encoding: each token is a uint32 = (arg << 8) | opcode with opcodes
 * LOAD=1 (push operand[arg][i]), SCALAR=2 (push scalars[arg] rounded once to
 * the compute type), ADD=3, SUB=4, MUL=5 (pop r, pop l, push l op r).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <string.h>

#define OR_LOAD 1u
#define OR_SCALAR 2u
#define OR_ADD 3u
#define OR_SUB 4u
#define OR_MUL 5u
#define OR_MAX_TOKENS 64
#define OR_MAX_STACK 64

/* Return codes: 0 ok, 1 bad program / argument. */

/* Host threads for the element-wise loops (1 unless set). */
static int g_threads = 1;

int oracle_set_threads(int t) {
    if (t < 1) return 1;
    g_threads = t;
    return 0;
}

int oracle_get_threads(void) { return g_threads; }

/* ---- program check (the oracle's own, minimal) ---------------------------- */
static int check_program(const uint32_t *prog, int len, int n_ops, int n_sc) {
    if (!prog || len <= 0 || len > OR_MAX_TOKENS) return 1;
    int depth = 0;
    for (int t = 0; t < len; ++t) {
        uint32_t op = prog[t] & 0xffu, arg = prog[t] >> 8;
        if (op == OR_LOAD) {
            if ((int)arg >= n_ops) return 1;
            ++depth;
        } else if (op == OR_SCALAR) {
            if ((int)arg >= n_sc) return 1;
            ++depth;
        } else if (op == OR_ADD || op == OR_SUB || op == OR_MUL) {
            if (arg != 0 || depth < 2) return 1;
            --depth;
        } else {
            return 1;
        }
        if (depth > OR_MAX_STACK) return 1;
    }
    return depth == 1 ? 0 : 1;
}

/* ---- 16-bit formats, from their definitions -------------------------------- */
static float f32_from_bits(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t bits_from_f32(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* bfloat16 is the upper half of a binary32 pattern: widening is exact. */
float oracle_bf16_to_f32(uint16_t h) { return f32_from_bits((uint32_t)h << 16); }

/* Round a binary32 to bfloat16, nearest-even. The 16 dropped bits decide:
 * above half rounds up, below half down, exactly half goes to the even
 * neighbour. A carry out of the significand bumps the exponent, and the
 * largest finite values round up to infinity, as IEEE rounding does. NaN stays
 * NaN (quiet, sign kept). */
uint16_t oracle_f32_to_bf16(float f) {
    uint32_t u = bits_from_f32(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)(((u >> 16) & 0x8000u) | 0x7fc0u);
    uint32_t kept = u >> 16, dropped = u & 0xffffu;
    if (dropped > 0x8000u || (dropped == 0x8000u && (kept & 1u))) ++kept;
    return (uint16_t)kept;
}

/* binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits. */
float oracle_f16_to_f32(uint16_t h) {
    uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    if (e == 0) {
        /* zero or subnormal: m * 2^-24, exact in binary32 */
        float v = ldexpf((float)m, -24);
        return sign ? -v : v;
    }
    if (e == 31) return f32_from_bits(sign | 0x7f800000u | (m << 13));
    return f32_from_bits(sign | ((e - 15u + 127u) << 23) | (m << 13));
}

/* Round a binary32 to binary16, nearest-even, with gradual underflow and
 * overflow to infinity. */
uint16_t oracle_f32_to_f16(float f) {
    uint32_t u = bits_from_f32(f);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    int32_t e = (int32_t)((u >> 23) & 0xffu);
    uint32_t m = u & 0x7fffffu;
    if (e == 255) return (uint16_t)(sign | (m ? 0x7e00u : 0x7c00u));
    int32_t E = e - 127 + 15; /* binary16 biased exponent of the value */
    if (E >= 31) return (uint16_t)(sign | 0x7c00u);
    if (E <= 0) {
        /* result is subnormal (or rounds up to the smallest normal): value is
         * sig * 2^(e-150), the binary16 subnormal step is 2^-24, so the
         * result is sig / 2^(126-e) rounded to an integer. */
        if (e == 0) return sign; /* binary32 subnormals are < 2^-126 */
        uint32_t sig = m | 0x800000u;
        int shift = 126 - e;
        if (shift >= 32) return sign;
        uint32_t q = sig >> shift, rem = sig & ((1u << shift) - 1u), half = 1u << (shift - 1);
        if (rem > half || (rem == half && (q & 1u))) ++q;
        return (uint16_t)(sign | q);
    }
    uint32_t q = ((uint32_t)E << 10) | (m >> 13), rem = m & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (q & 1u))) ++q; /* carry may reach inf: correct */
    return (uint16_t)(sign | q);
}

/* Array forms of the conversions above (kind 0 = bfloat16, 1 = binary16). */
void oracle_widen_h16(int kind, const uint16_t *h, double *out, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = (double)(kind == 0 ? oracle_bf16_to_f32(h[i]) : oracle_f16_to_f32(h[i]));
}

void oracle_narrow_h16(int kind, const float *f, uint16_t *out, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = kind == 0 ? oracle_f32_to_bf16(f[i]) : oracle_f32_to_f16(f[i]);
}

/* ---- element-wise evaluation: one stack machine run per element ----------- */

int oracle_eval_f64(const uint32_t *prog, int len, const double *const *ops, int n_ops,
                    const double *scalars, int n_sc, double *out, int64_t n) {
    if (check_program(prog, len, n_ops, n_sc) || n < 0) return 1;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n; ++i) {
        double st[OR_MAX_STACK];
        int sp = 0;
        for (int t = 0; t < len; ++t) {
            uint32_t op = prog[t] & 0xffu, arg = prog[t] >> 8;
            if (op == OR_LOAD) { st[sp++] = ops[arg][i]; continue; }
            if (op == OR_SCALAR) { st[sp++] = scalars[arg]; continue; }
            double r = st[--sp], l = st[--sp];
            st[sp++] = op == OR_ADD ? l + r : op == OR_SUB ? l - r : l * r;
        }
        out[i] = st[0];
    }
    return 0;
}

int oracle_eval_f32(const uint32_t *prog, int len, const float *const *ops, int n_ops,
                    const double *scalars, int n_sc, float *out, int64_t n) {
    if (check_program(prog, len, n_ops, n_sc) || n < 0) return 1;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n; ++i) {
        float st[OR_MAX_STACK];
        int sp = 0;
        for (int t = 0; t < len; ++t) {
            uint32_t op = prog[t] & 0xffu, arg = prog[t] >> 8;
            if (op == OR_LOAD) { st[sp++] = ops[arg][i]; continue; }
            if (op == OR_SCALAR) { st[sp++] = (float)scalars[arg]; continue; }
            float r = st[--sp], l = st[--sp];
            st[sp++] = op == OR_ADD ? l + r : op == OR_SUB ? l - r : l * r;
        }
        out[i] = st[0];
    }
    return 0;
}

/* 16-bit storage: widen each loaded value, run the binary32 machine, narrow
 * the result once. kind 0 = bfloat16, 1 = binary16. */
int oracle_eval_h16(int kind, const uint32_t *prog, int len, const uint16_t *const *ops,
                    int n_ops, const double *scalars, int n_sc, uint16_t *out, int64_t n) {
    if (check_program(prog, len, n_ops, n_sc) || n < 0 || (kind != 0 && kind != 1)) return 1;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n; ++i) {
        float st[OR_MAX_STACK];
        int sp = 0;
        for (int t = 0; t < len; ++t) {
            uint32_t op = prog[t] & 0xffu, arg = prog[t] >> 8;
            if (op == OR_LOAD) {
                uint16_t h = ops[arg][i];
                st[sp++] = kind == 0 ? oracle_bf16_to_f32(h) : oracle_f16_to_f32(h);
                continue;
            }
            if (op == OR_SCALAR) { st[sp++] = (float)scalars[arg]; continue; }
            float r = st[--sp], l = st[--sp];
            st[sp++] = op == OR_ADD ? l + r : op == OR_SUB ? l - r : l * r;
        }
        out[i] = kind == 0 ? oracle_f32_to_bf16(st[0]) : oracle_f32_to_f16(st[0]);
    }
    return 0;
}

/* ---- axpy: y <- alpha*x + y, alpha rounded once to the compute type ------- */

int oracle_axpy_f64(int64_t n, double alpha, const double *x, double *y) {
    if (n < 0) return 1;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n; ++i) y[i] = alpha * x[i] + y[i];
    return 0;
}

int oracle_axpy_f32(int64_t n, double alpha, const float *x, float *y) {
    if (n < 0) return 1;
    float a = (float)alpha;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n; ++i) y[i] = a * x[i] + y[i];
    return 0;
}

/* ---- reductions ------------------------------------------------------------ */

/* Error-free transformations (Ogita-Rump-Oishi 2005, Sec. 3): a product split
 * into its rounded value and exact error with one fused multiply-add, and a
 * sum split into its rounded value and exact error (Knuth's TwoSum). */
static void two_product(double a, double b, double *p, double *e) {
    *p = a * b;
    *e = fma(a, b, -*p);
}
static void two_sum(double a, double b, double *s, double *e) {
    *s = a + b;
    double z = *s - a;
    *e = (a - (*s - z)) + (b - z);
}

/* Dot2: the running sum p is carried with its accumulated rounding errors s,
 * which collect the exact error of every product and of every addition; the
 * result is p + s. Also returns sum |x_i y_i| (the tolerance scale). */
int oracle_dot2(int64_t n, const double *x, const double *y, double *result, double *abs_sum) {
    if (n < 0) return 1;
    double p = 0.0, s = 0.0, a = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double h, r, q;
        two_product(x[i], y[i], &h, &r);
        two_sum(p, h, &p, &q);
        s = s + (q + r);
        a = a + fabs(x[i] * y[i]);
    }
    *result = p + s;
    if (abs_sum) *abs_sum = a;
    return 0;
}

/* The unscaled 2-norm: square root of Dot2(x, x). */
int oracle_nrm2(int64_t n, const double *x, double *result) {
    double s;
    if (oracle_dot2(n, x, x, &s, 0)) return 1;
    *result = sqrt(s);
    return 0;
}

/* Plain sequential loops: CPU timing baseline and same-precision FP32 mode. */
double oracle_naive_dot_f64(int64_t n, const double *x, const double *y) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];
    return s;
}

float oracle_naive_dot_f32(int64_t n, const float *x, const float *y) {
    float s = 0.0f;
    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];
    return s;
}

/* Thread t of T owns elements [t*n/T, (t+1)*n/T) and sums them in order;
 * the partials are then added in thread order. *used gets the number of
 * threads that ran. The value depends on T (and equals the sequential loop's
 * for T = 1). */
double oracle_naive_dot_f64_par(int64_t n, const double *x, const double *y, int threads, int *used) {
    if (threads < 1) threads = 1;
    double part[256];
    if (threads > 256) threads = 256;
    int ran = 1;
#pragma omp parallel num_threads(threads) if (threads > 1)
    {
        const int T = omp_get_num_threads(), t = omp_get_thread_num();
        if (t == 0) ran = T;
        const int64_t lo = (int64_t)((__int128)n * t / T), hi = (int64_t)((__int128)n * (t + 1) / T);
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s = s + x[i] * y[i];
        part[t] = s;
    }
    double s = 0.0;
    for (int t = 0; t < ran; ++t) s = s + part[t];
    if (used) *used = ran;
    return s;
}

/* Copy nbytes with each of `threads` threads writing one contiguous share, so
 * that a fresh destination is first touched by the same split the parallel
 * loops above use. */
void oracle_parallel_copy(void *dst, const void *src, int64_t nbytes, int threads) {
    if (threads < 1) threads = 1;
#pragma omp parallel num_threads(threads) if (threads > 1)
    {
        const int T = omp_get_num_threads(), t = omp_get_thread_num();
        const int64_t lo = (int64_t)((__int128)nbytes * t / T), hi = (int64_t)((__int128)nbytes * (t + 1) / T);
        memcpy((char *)dst + lo, (const char *)src + lo, (size_t)(hi - lo));
    }
}

/* ---- the canonical summation order (second reduction oracle) -------------- */

/* The order, for storage type k with V = 16 / (element bytes) elements per
 * 16-byte chunk (V = 2, 4, 8 for binary64, binary32, 16-bit):
 *  1. tiles of T = 256 * 16 * V elements; elements past n read as zero;
 *  2. in tile t, "lane" l (0..255) visits chunks 16*256*t + 256*j + l for
 *     j = 0..15 in that order, and element p of a chunk (index chunk*V + p)
 *     goes to its slot p;
 *  3. a slot accumulates, for binary64, s = fma(x, y, s); for binary32,
 *     compensated binary32: p = x*y with its exact error fma(x, y, -p),
 *     TwoSum(s, p) -> (s, e), c = c + (e + product error); for 16-bit
 *     storage (exact binary32 products) TwoSum(s, x*y) -> (s, e), c = c + e;
 *     a slot's value is s (binary64) or (double)s + (double)c;
 *  4. the lane's value is the binary64 sum of its slot values in slot order;
 *  5. lanes form 4 groups of 64; a group is summed by a butterfly: for
 *     d = 1, 2, 4, ..., 32, every member i becomes v_i + v_(i xor d); the
 *     tile's partial is (g0 + g1) + (g2 + g3);
 *  6. the partials are combined by 1024 "lanes": lane l adds partials l,
 *     l + 1024, ... in order (from +0), the 16 groups of 64 lanes are summed
 *     by the same butterfly, and the 16 group sums by a pairwise tree
 *     (pairs (0,1), (2,3), ... then pairs of those, ...);
 *  7. nrm2 takes the square root; the result is rounded once to binary32
 *     for every storage type but binary64.
 * The value added per element is x*y (dot), x*x (nrm2) or |x|*1 (asum). */

#define RC_LANES 256
#define RC_CHUNKS 16
#define RC_FINAL 1024

static double rc_butterfly64(const double *v0) {
    double v[64], t[64];
    memcpy(v, v0, sizeof v);
    for (int d = 1; d < 64; d <<= 1) {
        for (int i = 0; i < 64; ++i) t[i] = v[i] + v[i ^ d];
        memcpy(v, t, sizeof v);
    }
    return v[0];
}

static void rc_two_sum_f(float a, float b, float *s, float *e) {
    *s = a + b;
    float z = *s - a;
    *e = (a - (*s - z)) + (b - z);
}

/* element i of a kind-k array as binary32 (kinds 1-3) */
static float rc_elem_f(int kind, const void *p, int64_t i) {
    if (kind == 1) return ((const float *)p)[i];
    uint16_t h = ((const uint16_t *)p)[i];
    return kind == 2 ? oracle_bf16_to_f32(h) : oracle_f16_to_f32(h);
}

static double rc_tile(int kind, int mode, int64_t n, const void *x, const void *y, int64_t t) {
    const int V = kind == 0 ? 2 : kind == 1 ? 4 : 8;
    double lane[RC_LANES];
    for (int l = 0; l < RC_LANES; ++l) {
        double sd[8];
        float sf[8], cf[8];
        for (int p = 0; p < 8; ++p) sd[p] = 0.0, sf[p] = 0.0f, cf[p] = 0.0f;
        for (int j = 0; j < RC_CHUNKS; ++j) {
            const int64_t chunk = t * RC_LANES * RC_CHUNKS + (int64_t)j * RC_LANES + l;
            for (int p = 0; p < V; ++p) {
                const int64_t i = chunk * V + p;
                if (kind == 0) {
                    double a = i < n ? ((const double *)x)[i] : 0.0, b;
                    if (mode == 0) b = i < n ? ((const double *)y)[i] : 0.0;
                    else if (mode == 1) b = a;
                    else a = fabs(a), b = 1.0;
                    sd[p] = fma(a, b, sd[p]);
                } else {
                    float a = i < n ? rc_elem_f(kind, x, i) : 0.0f, b, e;
                    if (mode == 0) b = i < n ? rc_elem_f(kind, y, i) : 0.0f;
                    else if (mode == 1) b = a;
                    else a = fabsf(a), b = 1.0f;
                    const float prod = a * b;
                    rc_two_sum_f(sf[p], prod, &sf[p], &e);
                    if (kind == 1) cf[p] = cf[p] + (e + fmaf(a, b, -prod));
                    else cf[p] = cf[p] + e;
                }
            }
        }
        double v = 0.0;
        for (int p = 0; p < V; ++p) {
            const double slot = kind == 0 ? sd[p] : (double)sf[p] + (double)cf[p];
            v = p == 0 ? slot : v + slot;
        }
        lane[l] = v;
    }
    double g[4];
    for (int k = 0; k < 4; ++k) g[k] = rc_butterfly64(lane + 64 * k);
    return (g[0] + g[1]) + (g[2] + g[3]);
}

/* kind: 0 binary64, 1 binary32, 2 bfloat16, 3 binary16 (raw bits);
 * mode: 0 dot, 1 nrm2, 2 asum (y unused for 1 and 2). The result is
 * written as binary64 (kind 0) or as the binary32 value widened. */
int oracle_reduce_canonical(int kind, int mode, int64_t n, const void *x, const void *y, double *result) {
    if (kind < 0 || kind > 3 || mode < 0 || mode > 2 || n < 0 || !result) return 1;
    const int V = kind == 0 ? 2 : kind == 1 ? 4 : 8;
    const int64_t T = (int64_t)RC_LANES * RC_CHUNKS * V;
    const int64_t P = (n + T - 1) / T;
    double fin[RC_FINAL];
    for (int l = 0; l < RC_FINAL; ++l) fin[l] = 0.0;
    /* partials are produced in tile order and folded straight into lane
     * (tile mod 1024), which is the order lane l adds them in */
    for (int64_t t = 0; t < P; ++t) fin[t % RC_FINAL] = fin[t % RC_FINAL] + rc_tile(kind, mode, n, x, y, t);
    double g[RC_FINAL / 64];
    for (int k = 0; k < RC_FINAL / 64; ++k) g[k] = rc_butterfly64(fin + 64 * k);
    for (int h = RC_FINAL / 128; h >= 1; h >>= 1)
        for (int k = 0; k < h; ++k) g[k] = g[2 * k] + g[2 * k + 1];
    double r = g[0];
    if (mode == 1) r = sqrt(r);
    *result = kind == 0 ? r : (double)(float)r;
    return 0;
}

/* ---- BLAS level-1 with increments ------------------------------------------ */

/* Offset (in elements) of element i of an n-element BLAS vector with
 * increment inc: i*inc for inc >= 0, (n-1-i)*|inc| for inc < 0. */
static int64_t blas_offset(int64_t i, int64_t n, int64_t inc) {
    return inc >= 0 ? i * inc : (n - 1 - i) * (-inc);
}

/* y_i <- x_i for i < n, elements of `esize` bytes, copied byte for byte. */
int oracle_copy(int64_t n, const void *x, int64_t incx, void *y, int64_t incy, int esize) {
    if (n < 0 || esize <= 0) return 1;
    for (int64_t i = 0; i < n; ++i)
        memcpy((char *)y + blas_offset(i, n, incy) * esize, (const char *)x + blas_offset(i, n, incx) * esize,
               (size_t)esize);
    return 0;
}

/* Index (from 0) of the first element of largest magnitude, scanning in
 * order and replacing the candidate only on a strictly larger magnitude, as
 * the reference BLAS does: a NaN never replaces the candidate, so a NaN is
 * the answer only when it is element 0. Returns -1 when n < 1 or inc <= 0
 * (the reference returns 0, its "no element", for these). */
int64_t oracle_iamax_f64(int64_t n, const double *x, int64_t inc) {
    if (n < 1 || inc <= 0) return -1;
    int64_t best = 0;
    double m = fabs(x[0]);
    for (int64_t i = 1; i < n; ++i) {
        const double a = fabs(x[i * inc]);
        if (a > m) {
            best = i;
            m = a;
        }
    }
    return best;
}

/* The same on binary32 values (16-bit storage is widened first, exactly). */
int64_t oracle_iamax_f32(int64_t n, const float *x, int64_t inc) {
    if (n < 1 || inc <= 0) return -1;
    int64_t best = 0;
    float m = fabsf(x[0]);
    for (int64_t i = 1; i < n; ++i) {
        const float a = fabsf(x[i * inc]);
        if (a > m) {
            best = i;
            m = a;
        }
    }
    return best;
}
