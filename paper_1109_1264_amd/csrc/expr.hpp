// expr.hpp -- compile-time expression trees and the catalogue of trees that
// get their own ahead-of-time kernels.
//
// A node type is the paper's expression-template node (Sec. 2, Fig. 1;
// node interface Sec. 4.2): it knows its postfix form (used on the host to
// match run-time programs against the catalogue) and evaluates itself for one
// element from a context that supplies operand values and scalars. All of a
// tree's evaluation is inlined into one kernel, so intermediates live in
// registers (the loop fusion of Sec. 2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "salt.h"

namespace salt {

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int K>
struct Ld {
    static constexpr int len = 1, n_loads = K + 1, n_scal = 0;
    static constexpr void emit(uint32_t *o, int &p) { o[p++] = SALT_TOKEN(SALT_OP_LOAD, K); }
    template <class G>
    __device__ __forceinline__ static auto ev(const G &g) { return g.template ld<K>(); }
};

template <int J>
struct Sc {
    static constexpr int len = 1, n_loads = 0, n_scal = J + 1;
    static constexpr void emit(uint32_t *o, int &p) { o[p++] = SALT_TOKEN(SALT_OP_SCALAR, J); }
    template <class G>
    __device__ __forceinline__ static auto ev(const G &g) { return g.template sc<J>(); }
};

template <int OP, class A, class B>
struct Bin {
    static constexpr int len = A::len + B::len + 1;
    static constexpr int n_loads = cmax(A::n_loads, B::n_loads);
    static constexpr int n_scal = cmax(A::n_scal, B::n_scal);
    static constexpr void emit(uint32_t *o, int &p) {
        A::emit(o, p);
        B::emit(o, p);
        o[p++] = SALT_TOKEN(OP, 0);
    }
    template <class G>
    __device__ __forceinline__ static auto ev(const G &g) {
        const auto l = A::ev(g);
        const auto r = B::ev(g);
        if constexpr (OP == SALT_OP_ADD) return l + r;
        else if constexpr (OP == SALT_OP_SUB) return l - r;
        else return l * r;
    }
};

template <class A, class B> using Add = Bin<SALT_OP_ADD, A, B>;
template <class A, class B> using Sub = Bin<SALT_OP_SUB, A, B>;
template <class A, class B> using Mul = Bin<SALT_OP_MUL, A, B>;

// The catalogue: trees written in canonical numbering (operands and scalars
// numbered in order of first appearance in postfix order).
//   copy     d = a                      (the bandwidth ceiling: 1 read, 1 write)
//   scale    d = alpha*a                (xSCAL out of place, Sec. 5)
//   fig1     d = a + (b - c)            (Fig. 1)
//   axpy     d = alpha*x + y            (xAXPY, Sec. 5)
//   tree5    d = a*b + c*e - f          (five-operand sweep tree)
//   abc      d = alpha*a + (b - c)      (the batched instance tree)
//   t4       d = alpha*(a + b) - c*e    (served tree)
//   t5       d = ((a*b + c)*(e - f)) + alpha*g   (served tree)
#define SALT_CATALOGUE(X)                                                        \
    X(copy, Ld<0>)                                                               \
    X(scale, Mul<Sc<0>, Ld<0>>)                                                  \
    X(fig1, Add<Ld<0>, Sub<Ld<1>, Ld<2>>>)                                       \
    X(axpy, Add<Mul<Sc<0>, Ld<0>>, Ld<1>>)                                       \
    X(tree5, Sub<Add<Mul<Ld<0>, Ld<1>>, Mul<Ld<2>, Ld<3>>>, Ld<4>>)              \
    X(abc, Add<Mul<Sc<0>, Ld<0>>, Sub<Ld<1>, Ld<2>>>)                            \
    X(t4, Sub<Mul<Sc<0>, Add<Ld<0>, Ld<1>>>, Mul<Ld<2>, Ld<3>>>)                 \
    X(t5, Add<Mul<Add<Mul<Ld<0>, Ld<1>>, Ld<2>>, Sub<Ld<3>, Ld<4>>>, Mul<Sc<0>, Ld<5>>>)

namespace cat {
#define SALT_CAT_TYPE(name, ...) using name = __VA_ARGS__;
SALT_CATALOGUE(SALT_CAT_TYPE)
#undef SALT_CAT_TYPE
enum Id {
#define SALT_CAT_ID(name, ...) id_##name,
    SALT_CATALOGUE(SALT_CAT_ID)
#undef SALT_CAT_ID
    count
};
}  // namespace cat

// Route of a program: a catalogue id, or kRouteGeneric for the interpreter.
constexpr int kRouteGeneric = -1;

// The empty second tree of a norm: nrm2(P) is the pair (P, NoTree).
struct NoTree {
    static constexpr int len = 0, n_loads = 0, n_scal = 0;
    static constexpr void emit(uint32_t *, int &) {}
};

// Reductions of trees with their own ahead-of-time kernels (the lazy
// evaluation of a tree inside a dot product or a norm, Sec. 2): dot(P, Q),
// or nrm2(P) when Q is NoTree. Operands and scalars are numbered in order of
// first appearance in P, then in Q; any other pair runs on the interpreter.
namespace rcat {
struct dot_sum_diff {  // dot(a + b, a - b)
    using P = Add<Ld<0>, Ld<1>>;
    using Q = Sub<Ld<0>, Ld<1>>;
};
struct nrm2_diff {  // nrm2(a - b): the norm of a difference
    using P = Sub<Ld<0>, Ld<1>>;
    using Q = NoTree;
};
struct nrm2_axpy {  // nrm2(alpha*a + b): the norm of an axpy result
    using P = Add<Mul<Sc<0>, Ld<0>>, Ld<1>>;
    using Q = NoTree;
};
}  // namespace rcat
#define SALT_RCATALOGUE(X) X(dot_sum_diff) X(nrm2_diff) X(nrm2_axpy)

namespace rcat {
enum Id {
#define SALT_RCAT_ID(name) id_##name,
    SALT_RCATALOGUE(SALT_RCAT_ID)
#undef SALT_RCAT_ID
    count
};
}  // namespace rcat

}  // namespace salt
