"""CPU oracle for the SALT hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU product path (the package
``paper_1109_1264_amd``) never imports, links or runs anything here, and the
two share no code: the only common module is the seeded input generator
(``paper_1109_1264_amd.workloads``), which holds none of the method's
arithmetic.

The arithmetic lives in ``salt_oracle.c`` (plain C, built with gcc and
``-ffp-contract=off``). This module loads it and wraps it for numpy arrays:

- :func:`eval_program` -- the fused element-wise expression (paper Sec. 2,
  Fig. 1), a per-element stack machine over the postfix tree.
- :func:`axpy` -- ``y <- alpha*x + y`` (Sec. 5, xAXPY).
- :func:`dot2`, :func:`nrm2` -- the root reductions (Sec. 2 "dot product or
  norm", Sec. 4.2 reduction step), as Dot2 values (Ogita-Rump-Oishi 2005).
- :func:`naive_dot` -- plain sequential loops (timing baseline, FP32 mode);
  :func:`naive_dot_par` -- the binary64 loop on several host threads (the
  all-cores timing baseline; per-thread partials added in thread order).
- :func:`set_threads` -- host threads for the element-wise loops (results do
  not depend on it: each element is computed alone).

16-bit storage arrays are ``numpy.uint16`` bit patterns; ``dtype`` names are
``"f64"``, ``"f32"``, ``"bf16"`` and ``"f16"``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "salt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# Opcodes of the postfix encoding (token = (arg << 8) | opcode). The oracle
# keeps its own copy: it shares no header with the GPU library.
LOAD, SCALAR, ADD, SUB, MUL = 1, 2, 3, 4, 5

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-fexcess-precision=standard"]


def build(force: bool = True) -> str:
    """Compile ``salt_oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded oracle library (built on first use if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = load(_LIB_PATH)
    return _lib


def load(path: str) -> ctypes.CDLL:
    """Load an oracle build from ``path`` and declare its signatures."""
    L = ctypes.CDLL(path)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    L.oracle_eval_f64.argtypes = [P, I, P, I, P, I, P, I64]
    L.oracle_eval_f32.argtypes = [P, I, P, I, P, I, P, I64]
    L.oracle_eval_h16.argtypes = [I, P, I, P, I, P, I, P, I64]
    for f in (L.oracle_eval_f64, L.oracle_eval_f32, L.oracle_eval_h16):
        f.restype = I
    L.oracle_axpy_f64.argtypes = [I64, D, P, P]
    L.oracle_axpy_f32.argtypes = [I64, D, P, P]
    L.oracle_axpy_f64.restype = L.oracle_axpy_f32.restype = I
    L.oracle_dot2.argtypes = [I64, P, P, P, P]
    L.oracle_dot2.restype = I
    L.oracle_nrm2.argtypes = [I64, P, P]
    L.oracle_nrm2.restype = I
    L.oracle_naive_dot_f64.argtypes = [I64, P, P]
    L.oracle_naive_dot_f64.restype = D
    L.oracle_naive_dot_f32.argtypes = [I64, P, P]
    L.oracle_naive_dot_f32.restype = ctypes.c_float
    L.oracle_naive_dot_f64_par.argtypes = [I64, P, P, I, P]
    L.oracle_naive_dot_f64_par.restype = D
    L.oracle_parallel_copy.argtypes = [P, P, I64, I]
    L.oracle_parallel_copy.restype = None
    L.oracle_set_threads.argtypes = [I]
    L.oracle_set_threads.restype = I
    L.oracle_get_threads.argtypes = []
    L.oracle_get_threads.restype = I
    L.oracle_reduce_canonical.argtypes = [I, I, I64, P, P, P]
    L.oracle_reduce_canonical.restype = I
    L.oracle_copy.argtypes = [I64, P, I64, P, I64, I]
    L.oracle_copy.restype = I
    L.oracle_iamax_f64.argtypes = [I64, P, I64]
    L.oracle_iamax_f64.restype = I64
    L.oracle_iamax_f32.argtypes = [I64, P, I64]
    L.oracle_iamax_f32.restype = I64
    L.oracle_widen_h16.argtypes = [I, P, P, I64]
    L.oracle_widen_h16.restype = None
    L.oracle_narrow_h16.argtypes = [I, P, P, I64]
    L.oracle_narrow_h16.restype = None
    L.oracle_bf16_to_f32.argtypes = [ctypes.c_uint16]
    L.oracle_bf16_to_f32.restype = ctypes.c_float
    L.oracle_f32_to_bf16.argtypes = [ctypes.c_float]
    L.oracle_f32_to_bf16.restype = ctypes.c_uint16
    L.oracle_f16_to_f32.argtypes = [ctypes.c_uint16]
    L.oracle_f16_to_f32.restype = ctypes.c_float
    L.oracle_f32_to_f16.argtypes = [ctypes.c_float]
    L.oracle_f32_to_f16.restype = ctypes.c_uint16
    return L


_NP = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16, "f16": np.uint16}


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _ptr_array(arrays):
    arr = (ctypes.c_void_p * max(1, len(arrays)))()
    for k, a in enumerate(arrays):
        arr[k] = _ptr(a)
    return arr


def eval_program(prog, operands, scalars, dtype: str, n: int | None = None) -> np.ndarray:
    """Evaluate a postfix program element by element (see module docstring).

    ``operands`` are 1-D arrays of the storage type, ``scalars`` Python floats
    (rounded once to the compute type). Returns a new array of length ``n``.
    """
    prog = np.ascontiguousarray(prog, dtype=np.uint32)
    ops = [np.ascontiguousarray(a, dtype=_NP[dtype]) for a in operands]
    if n is None:
        n = len(ops[0]) if ops else 0
    for a in ops:
        if len(a) < n:
            raise ValueError("operand shorter than n")
    sc = np.ascontiguousarray(scalars, dtype=np.float64).reshape(-1)
    out = np.empty(n, dtype=_NP[dtype])
    L = lib()
    pa = _ptr_array(ops)
    scp = _ptr(sc) if len(sc) else None
    if dtype == "f64":
        rc = L.oracle_eval_f64(_ptr(prog), len(prog), pa, len(ops), scp, len(sc), _ptr(out), n)
    elif dtype == "f32":
        rc = L.oracle_eval_f32(_ptr(prog), len(prog), pa, len(ops), scp, len(sc), _ptr(out), n)
    else:
        kind = 0 if dtype == "bf16" else 1
        rc = L.oracle_eval_h16(kind, _ptr(prog), len(prog), pa, len(ops), scp, len(sc), _ptr(out), n)
    if rc != 0:
        raise ValueError("oracle rejected the program or arguments")
    return out


def axpy(alpha: float, x: np.ndarray, y: np.ndarray, dtype: str) -> np.ndarray:
    """Return ``alpha*x + y`` (a new array; ``y`` is not modified)."""
    x = np.ascontiguousarray(x, dtype=_NP[dtype])
    out = np.array(y, dtype=_NP[dtype], copy=True)
    L = lib()
    if dtype == "f64":
        L.oracle_axpy_f64(len(x), float(alpha), _ptr(x), _ptr(out))
    elif dtype == "f32":
        L.oracle_axpy_f32(len(x), float(alpha), _ptr(x), _ptr(out))
    else:
        # 16-bit storage: the axpy tree through the generic 16-bit machine.
        return eval_program([(0 << 8) | SCALAR, (0 << 8) | LOAD, MUL, (1 << 8) | LOAD, ADD],
                            [x, out], [alpha], dtype)
    return out


def widen(a: np.ndarray, dtype: str) -> np.ndarray:
    """Exact value of stored elements as float64 (16-bit storage widened)."""
    if dtype in ("f64", "f32"):
        return np.asarray(a, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.uint16)
    out = np.empty(len(a), dtype=np.float64)
    lib().oracle_widen_h16(0 if dtype == "bf16" else 1, _ptr(a), _ptr(out), len(a))
    return out


def narrow(values, dtype: str) -> np.ndarray:
    """Round binary32 values to 16-bit storage with the oracle's RNE rule."""
    f = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
    out = np.empty(len(f), dtype=np.uint16)
    lib().oracle_narrow_h16(0 if dtype == "bf16" else 1, _ptr(f), _ptr(out), len(f))
    return out


def dot2(x: np.ndarray, y: np.ndarray) -> tuple[float, float]:
    """Dot2 value of sum x_i*y_i in binary64, and sum |x_i*y_i|.

    Inputs must already be float64 (use :func:`widen` for stored values).
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    if len(x) != len(y):
        raise ValueError("length mismatch")
    r = ctypes.c_double()
    a = ctypes.c_double()
    lib().oracle_dot2(len(x), _ptr(x), _ptr(y), ctypes.byref(r), ctypes.byref(a))
    return r.value, a.value


def nrm2(x: np.ndarray) -> float:
    """sqrt(Dot2(x, x)) of float64 values."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = ctypes.c_double()
    lib().oracle_nrm2(len(x), _ptr(x), ctypes.byref(r))
    return r.value


def naive_dot(x: np.ndarray, y: np.ndarray, dtype: str = "f64") -> float:
    """Plain sequential loop in binary64 or binary32."""
    L = lib()
    if dtype == "f32":
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        return float(L.oracle_naive_dot_f32(len(x), _ptr(x), _ptr(y)))
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return float(L.oracle_naive_dot_f64(len(x), _ptr(x), _ptr(y)))


def naive_dot_par(x: np.ndarray, y: np.ndarray, threads: int) -> tuple[float, int]:
    """The binary64 loop split over ``threads`` host threads: thread t sums
    elements [t*n/T, (t+1)*n/T) in order, the partials are added in thread
    order. Returns the sum and the number of threads that ran."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    if len(x) != len(y):
        raise ValueError("length mismatch")
    used = ctypes.c_int(0)
    r = lib().oracle_naive_dot_f64_par(len(x), _ptr(x), _ptr(y), int(threads), ctypes.byref(used))
    return float(r), used.value


def set_threads(threads: int) -> None:
    """Host threads for the element-wise loops (eval, axpy)."""
    if lib().oracle_set_threads(int(threads)) != 0:
        raise ValueError("threads must be >= 1")


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def first_touch_copy(a: np.ndarray, threads: int) -> np.ndarray:
    """A copy of ``a`` in fresh memory written by ``threads`` threads, each
    one contiguous share (so its pages sit near the thread that uses them)."""
    a = np.ascontiguousarray(a)
    out = np.empty_like(a)
    lib().oracle_parallel_copy(_ptr(out), _ptr(a), a.nbytes, int(threads))
    return out


_KIND = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
MODES = {"dot": 0, "nrm2": 1, "asum": 2}


def reduce_canonical(mode: str, x: np.ndarray, y: np.ndarray | None, dtype: str):
    """dot / nrm2 / asum of stored values in the library's documented
    summation order (tiles of 256 lanes x 16 chunks, per-slot accumulators,
    butterflies, a 1024-lane combine; the order is a reading, since the
    paper leaves it open). Returns np.float64 for binary64 storage, else
    np.float32 -- the result type, for bit-for-bit comparison."""
    x = np.ascontiguousarray(x, dtype=_NP[dtype])
    yy = x if y is None else np.ascontiguousarray(y, dtype=_NP[dtype])
    if mode == "dot" and len(yy) != len(x):
        raise ValueError("length mismatch")
    r = ctypes.c_double()
    if lib().oracle_reduce_canonical(_KIND[dtype], MODES[mode], len(x), _ptr(x), _ptr(yy), ctypes.byref(r)):
        raise ValueError("bad arguments")
    return np.float64(r.value) if dtype == "f64" else np.float32(r.value)


# ---------------------------------------------------------------------------
# BLAS level-1 with increments (reference BLAS conventions): element i of an
# n-element vector with increment inc is x[i*inc] (inc >= 0) or
# x[(n-1-i)*|inc|] (inc < 0). The strided operations are gathers into
# contiguous vectors, the contiguous definitions above, and a scatter back.
# ---------------------------------------------------------------------------

def blas_span(n: int, inc: int) -> int:
    """Elements an n-element vector with increment inc spans (>= 1 if n > 0)."""
    return 0 if n <= 0 else 1 + (n - 1) * abs(inc)


def copy(n: int, x: np.ndarray, incx: int, y: np.ndarray, incy: int) -> np.ndarray:
    """Return a copy of ``y`` with y_i <- x_i (byte for byte)."""
    x = np.ascontiguousarray(x)
    out = np.array(y, copy=True)
    if x.dtype.itemsize != out.dtype.itemsize:
        raise ValueError("element sizes differ")
    if n > 0 and (len(x) < blas_span(n, incx) or len(out) < blas_span(n, incy)):
        raise ValueError("array shorter than the strided vector")
    if lib().oracle_copy(n, _ptr(x), incx, _ptr(out), incy, out.dtype.itemsize) != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def gather(n: int, x: np.ndarray, inc: int) -> np.ndarray:
    """The n elements of a strided vector, contiguous, in element order."""
    x = np.ascontiguousarray(x)
    return copy(n, x, inc, np.empty(max(n, 0), dtype=x.dtype), 1)


def scatter(n: int, v: np.ndarray, y: np.ndarray, inc: int) -> np.ndarray:
    """Return a copy of ``y`` with its strided elements replaced by ``v``."""
    return copy(n, np.ascontiguousarray(v, dtype=np.asarray(y).dtype), 1, y, inc)


def scal(n: int, alpha: float, x: np.ndarray, inc: int, dtype: str) -> np.ndarray:
    """x_i <- alpha*x_i (a new array). inc <= 0: unchanged (reference BLAS)."""
    x = np.array(x, dtype=_NP[dtype], copy=True)
    if n <= 0 or inc <= 0:
        return x
    v = eval_program([(0 << 8) | SCALAR, (0 << 8) | LOAD, MUL], [gather(n, x, inc)], [alpha], dtype)
    return scatter(n, v, x, inc)


def axpy_strided(n: int, alpha: float, x: np.ndarray, incx: int, y: np.ndarray, incy: int,
                 dtype: str) -> np.ndarray:
    """y_i <- alpha*x_i + y_i (a new array)."""
    y = np.array(y, dtype=_NP[dtype], copy=True)
    if n <= 0:
        return y
    v = axpy(alpha, gather(n, np.asarray(x, dtype=_NP[dtype]), incx), gather(n, y, incy), dtype)
    return scatter(n, v, y, incy)


def asum(x: np.ndarray) -> tuple[float, float]:
    """sum |x_i| of float64 values (Dot2 against ones), and the same value as
    the tolerance scale."""
    a = np.abs(np.ascontiguousarray(x, dtype=np.float64))
    r, s = dot2(a, np.ones(len(a)))
    return r, s


def iamax(n: int, x: np.ndarray, inc: int, dtype: str) -> int:
    """Index (from 0) of the first element of largest magnitude; -1 when
    n < 1 or inc <= 0. 16-bit storage is compared on its exact binary32
    values."""
    if n < 1 or inc <= 0:
        return -1
    if len(x) < blas_span(n, inc):
        raise ValueError("array shorter than the strided vector")
    L = lib()
    if dtype == "f64":
        a = np.ascontiguousarray(x, dtype=np.float64)
        return int(L.oracle_iamax_f64(n, _ptr(a), inc))
    a = np.ascontiguousarray(x, dtype=np.float32) if dtype == "f32" else widen(x, dtype).astype(np.float32)
    return int(L.oracle_iamax_f32(n, _ptr(a), inc))


# Reduction tolerances, relative to sum |x_i*y_i| of the stored values.
TOL = {"f64": 1e-13, "f32": 1e-6, "bf16": 1e-6, "f16": 1e-6}
