"""Thin ctypes binding of ``libsalt.so`` (include/salt.h), same names.

Only argument marshalling happens here: torch tensors are turned into device
pointers and the current HIP stream, and every computation runs in the
library's kernels. There is no fallback: if the library is missing the first
call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsalt.so")

# Element types and status codes (include/salt.h).
F64, F32, BF16, F16 = 0, 1, 2, 3
OK, ERR_ARG, ERR_PROGRAM, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_DEVICE = range(6)
LOAD, SCALAR, ADD, SUB, MUL = 1, 2, 3, 4, 5
MAX_TOKENS, MAX_OPERANDS, MAX_SCALARS, MAX_STACK = 64, 8, 8, 8

DTYPE_NAMES = {F64: "f64", F32: "f32", BF16: "bf16", F16: "f16"}
ELEM_BYTES = {F64: 8, F32: 4, BF16: 2, F16: 2}


def token(op: int, arg: int = 0) -> int:
    return ((arg << 8) | op) & 0xFFFFFFFF


class SaltError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("salt status %d (%s): %s" % (status, _status_string(status), message))
        self.status = status


class LaunchConfig(ctypes.Structure):
    """salt_launch_config: unroll (0 = tuned), nontemporal (-1 = tuned),
    blocks (-1 = tuned, 0 = one workgroup per tile)."""
    _fields_ = [("unroll", ctypes.c_int32), ("nontemporal", ctypes.c_int32), ("blocks", ctypes.c_int64)]

    def __init__(self, unroll=0, nontemporal=-1, blocks=-1):
        super().__init__(unroll, nontemporal, blocks)

    def as_tuple(self):
        return (self.unroll, self.nontemporal, self.blocks)


class BatchItem(ctypes.Structure):
    """salt_batch_item."""
    _fields_ = [("n", ctypes.c_int64), ("operands", ctypes.c_void_p * MAX_OPERANDS),
                ("scalars", ctypes.c_double * MAX_SCALARS), ("out", ctypes.c_void_p),
                ("dot_out", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsalt.so and declare its C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsalt.so is not built (run python -m paper_1109_1264_amd.build)")
    # torch brings its own HIP runtime; loading it first makes libsalt bind to
    # that same runtime, so device pointers and streams are shared. Loading
    # libsalt first would start a second HIP runtime in the process.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise RuntimeError("two HIP runtimes are loaded (%s): libsalt must share torch's" % sorted(runtimes))
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    U32P = ctypes.POINTER(ctypes.c_uint32)
    CFG = ctypes.POINTER(LaunchConfig)
    sigs = {
        "salt_eval": ([U32P, I32, P, I32, P, I32, P, I64, I32, P], I32),
        "salt_eval_ex": ([U32P, I32, P, I32, P, I32, P, I64, I32, P, CFG], I32),
        "salt_axpy": ([I64, D, P, P, I32, P], I32),
        "salt_reduce_workspace_bytes": ([I64, I32], SZ),
        "salt_reduce_tile_elems": ([I32], I64),
        "salt_dot": ([I64, P, P, P, P, SZ, I32, P], I32),
        "salt_dot_ex": ([I64, P, P, P, P, SZ, I32, P, CFG], I32),
        "salt_dot_noalloc": ([I64, P, P, P, I32, P], I32),
        "salt_stream_reference": ([I32, I32, P, P, I64, P], I32),
        "salt_nrm2": ([I64, P, P, P, SZ, I32, P], I32),
        "salt_nrm2_ex": ([I64, P, P, P, SZ, I32, P, CFG], I32),
        "salt_reduce_partials": ([I32, I64, P, P, P, I32, P], I32),
        "salt_reduce_combine": ([I32, P, I64, P, I32, P], I32),
        "salt_scal": ([I64, D, P, I64, I32, P], I32),
        "salt_copy": ([I64, P, I64, P, I64, I32, P], I32),
        "salt_axpy_strided": ([I64, D, P, I64, P, I64, I32, P], I32),
        "salt_dot_strided": ([I64, P, I64, P, I64, P, P, SZ, I32, P], I32),
        "salt_nrm2_strided": ([I64, P, I64, P, P, SZ, I32, P], I32),
        "salt_asum": ([I64, P, I64, P, P, SZ, I32, P], I32),
        "salt_iamax": ([I64, P, I64, P, P, SZ, I32, P], I32),
        "salt_tuning_load": ([ctypes.c_char_p], I32),
        "salt_tuning_lookup": ([I32, I32, I32, I64, CFG], I32),
        "salt_catalogue_count": ([], I32),
        "salt_catalogue_program": ([I32, U32P, I32, ctypes.POINTER(ctypes.c_char_p)], I32),
        "salt_program_route": ([U32P, I32, I32, I32, ctypes.POINTER(I32)], I32),
        "salt_reduce_expr_route": ([U32P, I32, U32P, I32, I32, I32, I32, ctypes.POINTER(I32)], I32),
        "salt_jit_compile_reduce": ([U32P, I32, U32P, I32, I32, I32, I32], I32),
        "salt_eval_chunking": ([I32, I64, I32, ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
        "salt_jit_code_reduce": ([U32P, I32, U32P, I32, I32, I32, I32, P, SZ, ctypes.POINTER(SZ)], I32),
        "salt_jit_set_mode": ([I32], I32),
        "salt_jit_compile": ([U32P, I32, I32, I32, I32], I32),
        "salt_jit_code": ([U32P, I32, I32, I32, I32, P, SZ, ctypes.POINTER(SZ)], I32),
        "salt_eval_route": ([U32P, I32, I32, I32, I32, ctypes.POINTER(I32)], I32),
        "salt_program_check": ([U32P, I32, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)], I32),
        "salt_status_string": ([I32], ctypes.c_char_p),
        "salt_last_error": ([], ctypes.c_char_p),
        "salt_version": ([], I32),
        "salt_dot_expr": ([U32P, I32, U32P, I32, P, I32, P, I32, I64, P, P, SZ, I32, P], I32),
        "salt_nrm2_expr": ([U32P, I32, P, I32, P, I32, I64, P, P, SZ, I32, P], I32),
        "salt_dot_expr_ex": ([U32P, I32, U32P, I32, P, I32, P, I32, I64, P, P, SZ, I32, P, CFG], I32),
        "salt_nrm2_expr_ex": ([U32P, I32, P, I32, P, I32, I64, P, P, SZ, I32, P, CFG], I32),
        "salt_batch_plan_create": ([U32P, I32, I32, I32, ctypes.POINTER(BatchItem), I32, I32,
                                    ctypes.POINTER(P)], I32),
        "salt_batch_plan_info": ([P, ctypes.POINTER(SZ), ctypes.POINTER(SZ), ctypes.POINTER(I64)], I32),
        "salt_batch_upload": ([P, P, SZ, P], I32),
        "salt_batch_launch": ([P, P, SZ, P, CFG], I32),
        "salt_batch_graph_create": ([P, P, SZ, CFG, ctypes.POINTER(P)], I32),
        "salt_graph_launch": ([P, P], I32),
        "salt_graph_destroy": ([P], None),
        "salt_batch_plan_destroy": ([P], None),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _hip_runtimes_mapped() -> set:
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as fh:
            return {l.split()[-1] for l in fh if "libamdhip64" in l}
    except OSError:
        return set()


def _status_string(s: int) -> str:
    try:
        return lib().salt_status_string(s).decode()
    except Exception:  # pragma: no cover - only used in error text
        return "?"


def check(status: int) -> None:
    if status != OK:
        raise SaltError(status, lib().salt_last_error().decode())


_PROGS = {}  # token tuple -> (ctypes array, length); the library only reads it


def _prog(tokens: Sequence[int]):
    key = tuple(tokens)
    hit = _PROGS.get(key)
    if hit is None:
        if len(_PROGS) >= 4096:
            _PROGS.clear()
        hit = ((ctypes.c_uint32 * max(1, len(key)))(*[int(t) & 0xFFFFFFFF for t in key]), len(key))
        _PROGS[key] = hit
    return hit


# ---------------------------------------------------------------------------
# torch plumbing (device memory and streams only)
# ---------------------------------------------------------------------------

_CODES = {}


def dtype_code(t) -> int:
    if not _CODES:
        import torch

        _CODES.update({torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16})
    c = _CODES.get(t.dtype)
    if c is None:
        raise TypeError("unsupported tensor dtype %s" % t.dtype)
    return c


def _stream_ptr(stream) -> int:
    import torch

    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:  # the current stream's handle without a Stream object
            return int(raw(torch._C._cuda_getDevice()))
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _dev(t):
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if t.dim() != 1 or (t.numel() > 1 and t.stride(0) != 1):
        raise ValueError("tensors must be contiguous 1-D vectors")
    return t.data_ptr()


def _cfg(config):
    if config is None:
        return None
    if isinstance(config, LaunchConfig):
        return ctypes.byref(config)
    return ctypes.byref(LaunchConfig(*config))


def salt_eval(prog: Sequence[int], operands, scalars, out, n: int | None = None,
              stream=None, config=None) -> None:
    """out[i] = prog(operands[...][i]; scalars) on the GPU (see salt.h)."""
    d = dtype_code(out)
    if n is None:
        n = out.numel()
    if out.numel() < n:
        raise ValueError("tensor shorter than n")
    ptrs = []
    for t in operands:
        if dtype_code(t) != d:
            raise TypeError("all operands must have the output's dtype")
        if t.numel() < n:
            raise ValueError("tensor shorter than n")
        ptrs.append(_dev(t))
    parr, plen = _prog(prog)
    ops = (ctypes.c_void_p * max(1, len(ptrs)))(*ptrs)
    sc = (ctypes.c_double * max(1, len(scalars)))(*[float(s) for s in scalars])
    L = lib()
    if config is None:
        st = L.salt_eval(parr, plen, ops, len(operands), sc, len(scalars), _dev(out), n, d, _stream_ptr(stream))
    else:
        st = L.salt_eval_ex(parr, plen, ops, len(operands), sc, len(scalars), _dev(out), n, d,
                            _stream_ptr(stream), _cfg(config))
    check(st)


def salt_axpy(alpha: float, x, y, n: int | None = None, stream=None) -> None:
    """y <- alpha*x + y."""
    d = dtype_code(y)
    if dtype_code(x) != d:
        raise TypeError("x and y must share a dtype")
    if n is None:
        n = y.numel()
    if x.numel() < n or y.numel() < n:
        raise ValueError("tensor shorter than n")
    check(lib().salt_axpy(n, float(alpha), _dev(x), _dev(y), d, _stream_ptr(stream)))


def salt_reduce_workspace_bytes(n: int, dtype: int) -> int:
    return int(lib().salt_reduce_workspace_bytes(n, dtype))


def salt_reduce_tile_elems(dtype: int) -> int:
    return int(lib().salt_reduce_tile_elems(dtype))


def workspace(n: int, dtype: int, device="cuda"):
    """A device workspace of the size dot / nrm2 need for length n."""
    import torch

    nbytes = salt_reduce_workspace_bytes(n, dtype)
    return torch.empty(max(1, (nbytes + 7) // 8), dtype=torch.float64, device=device)


def _result_tensor(d, device):
    import torch

    return torch.empty(1, dtype=torch.float64 if d == F64 else torch.float32, device=device)


def salt_dot(x, y, n: int | None = None, result=None, ws=None, stream=None, config=None):
    """Device scalar sum x[i]*y[i] (binary64 for F64, else binary32)."""
    d = dtype_code(x)
    if dtype_code(y) != d:
        raise TypeError("x and y must share a dtype")
    if n is None:
        n = x.numel()
    if x.numel() < n or y.numel() < n:
        raise ValueError("tensor shorter than n")
    result = _result_tensor(d, x.device) if result is None else result
    ws = workspace(n, d, x.device) if ws is None else ws
    nb = ws.numel() * ws.element_size()
    L = lib()
    if config is None:
        st = L.salt_dot(n, _dev(x), _dev(y), _dev(result), _dev(ws), nb, d, _stream_ptr(stream))
    else:
        st = L.salt_dot_ex(n, _dev(x), _dev(y), _dev(result), _dev(ws), nb, d, _stream_ptr(stream), _cfg(config))
    check(st)
    return result


def salt_dot_noalloc(x, y, n: int | None = None, result=None, stream=None):
    """salt_dot with the library's own partials buffer (no workspace)."""
    d = dtype_code(x)
    if dtype_code(y) != d:
        raise TypeError("x and y must share a dtype")
    if n is None:
        n = x.numel()
    if x.numel() < n or y.numel() < n:
        raise ValueError("tensor shorter than n")
    result = _result_tensor(d, x.device) if result is None else result
    check(lib().salt_dot_noalloc(n, _dev(x), _dev(y), _dev(result), d, _stream_ptr(stream)))
    return result


def salt_stream_reference(inputs, out=None, nbytes: int | None = None, stream=None) -> None:
    """The plain read/write stream of the same name (a bandwidth reference):
    out = xor of the inputs, 16-byte chunks; out None reads only."""
    if nbytes is None:
        nbytes = inputs[0].numel() * inputs[0].element_size()
    arr = (ctypes.c_void_p * len(inputs))(*[t.data_ptr() for t in inputs])
    check(lib().salt_stream_reference(len(inputs), 0 if out is None else 1, arr,
                                      None if out is None else _dev(out), nbytes, _stream_ptr(stream)))


def salt_nrm2(x, n: int | None = None, result=None, ws=None, stream=None, config=None):
    """Device scalar sqrt(sum x[i]^2)."""
    d = dtype_code(x)
    if n is None:
        n = x.numel()
    if x.numel() < n:
        raise ValueError("tensor shorter than n")
    result = _result_tensor(d, x.device) if result is None else result
    ws = workspace(n, d, x.device) if ws is None else ws
    nb = ws.numel() * ws.element_size()
    L = lib()
    if config is None:
        st = L.salt_nrm2(n, _dev(x), _dev(result), _dev(ws), nb, d, _stream_ptr(stream))
    else:
        st = L.salt_nrm2_ex(n, _dev(x), _dev(result), _dev(ws), nb, d, _stream_ptr(stream), _cfg(config))
    check(st)
    return result


# ---------------------------------------------------------------------------
# sharded reductions: pass 1 per shard (shards split at tile boundaries),
# pass 2 over the partials placed side by side
# ---------------------------------------------------------------------------

MODE_DOT, MODE_NRM2, MODE_ASUM = 0, 1, 2


def salt_reduce_partials(mode: int, x, y=None, n: int | None = None, partials=None, stream=None):
    """Device float64 tensor of the ceil(n / tile) partials of one shard."""
    import torch

    d = dtype_code(x)
    if n is None:
        n = x.numel()
    if mode == MODE_DOT and (y is None or dtype_code(y) != d):
        raise TypeError("dot needs y of the same dtype")
    count = (n + salt_reduce_tile_elems(d) - 1) // salt_reduce_tile_elems(d)
    if partials is None:
        partials = torch.empty(max(count, 1), dtype=torch.float64, device=x.device)
    check(lib().salt_reduce_partials(mode, n, _dev(x), _dev(y) if y is not None else None, _dev(partials), d,
                                     _stream_ptr(stream)))
    return partials[:count]


def salt_reduce_combine(mode: int, partials, dtype: int, count: int | None = None, result=None, stream=None):
    """Device scalar from partials (the fixed pass-2 combine)."""
    if count is None:
        count = partials.numel()
    result = _result_tensor(dtype, partials.device) if result is None else result
    check(lib().salt_reduce_combine(mode, _dev(partials), count, _dev(result), dtype, _stream_ptr(stream)))
    return result


# ---------------------------------------------------------------------------
# BLAS level-1 with increments: a vector is (tensor, n, inc), element i at
# t[i*inc] (inc >= 0) or t[(n-1-i)*|inc|] (inc < 0); the tensor holds at
# least 1 + (n-1)*|inc| elements.
# ---------------------------------------------------------------------------

def _span(n: int, inc: int) -> int:
    return 0 if n <= 0 else 1 + (n - 1) * abs(inc)


def _strided(t, n: int, inc: int, name: str, needed: bool = True):
    if needed and n > 0 and t.numel() < _span(n, inc):
        raise ValueError("%s holds %d elements, the strided vector spans %d" % (name, t.numel(), _span(n, inc)))
    return _dev(t)


def salt_scal(alpha: float, x, n: int, incx: int = 1, stream=None) -> None:
    """x_i <- alpha*x_i (nothing for incx <= 0)."""
    check(lib().salt_scal(n, float(alpha), _strided(x, n, incx, "x", incx > 0), incx, dtype_code(x),
                          _stream_ptr(stream)))


def salt_copy(x, y, n: int, incx: int = 1, incy: int = 1, stream=None) -> None:
    """y_i <- x_i."""
    d = dtype_code(y)
    if dtype_code(x) != d:
        raise TypeError("x and y must share a dtype")
    check(lib().salt_copy(n, _strided(x, n, incx, "x"), incx, _strided(y, n, incy, "y"), incy, d,
                          _stream_ptr(stream)))


def salt_axpy_strided(alpha: float, x, y, n: int, incx: int = 1, incy: int = 1, stream=None) -> None:
    """y_i <- alpha*x_i + y_i."""
    d = dtype_code(y)
    if dtype_code(x) != d:
        raise TypeError("x and y must share a dtype")
    check(lib().salt_axpy_strided(n, float(alpha), _strided(x, n, incx, "x"), incx, _strided(y, n, incy, "y"),
                                  incy, d, _stream_ptr(stream)))


def _reduce_args(x, n, result, ws):
    d = dtype_code(x)
    result = _result_tensor(d, x.device) if result is None else result
    ws = workspace(n, d, x.device) if ws is None else ws
    return d, result, ws, ws.numel() * ws.element_size()


def salt_dot_strided(x, y, n: int, incx: int = 1, incy: int = 1, result=None, ws=None, stream=None):
    """Device scalar sum_i x_i*y_i over strided vectors."""
    if dtype_code(y) != dtype_code(x):
        raise TypeError("x and y must share a dtype")
    d, result, ws, nb = _reduce_args(x, n, result, ws)
    check(lib().salt_dot_strided(n, _strided(x, n, incx, "x"), incx, _strided(y, n, incy, "y"), incy,
                                 _dev(result), _dev(ws), nb, d, _stream_ptr(stream)))
    return result


def salt_nrm2_strided(x, n: int, incx: int = 1, result=None, ws=None, stream=None):
    """Device scalar sqrt(sum_i x_i^2) (0 for incx <= 0)."""
    d, result, ws, nb = _reduce_args(x, n, result, ws)
    check(lib().salt_nrm2_strided(n, _strided(x, n, incx, "x", incx > 0), incx, _dev(result), _dev(ws), nb, d,
                                  _stream_ptr(stream)))
    return result


def salt_asum(x, n: int | None = None, incx: int = 1, result=None, ws=None, stream=None):
    """Device scalar sum_i |x_i| (0 for incx <= 0)."""
    if n is None:
        n = x.numel()
    d, result, ws, nb = _reduce_args(x, n, result, ws)
    check(lib().salt_asum(n, _strided(x, n, incx, "x", incx > 0), incx, _dev(result), _dev(ws), nb, d,
                          _stream_ptr(stream)))
    return result


def salt_iamax(x, n: int | None = None, incx: int = 1, result=None, ws=None, stream=None):
    """Device int64: index (from 0) of the first element of largest magnitude;
    -1 for n < 1 or incx <= 0."""
    import torch

    if n is None:
        n = x.numel()
    d = dtype_code(x)
    result = torch.empty(1, dtype=torch.int64, device=x.device) if result is None else result
    if result.dtype != torch.int64:
        raise TypeError("result must be an int64 tensor")
    ws = workspace(n, d, x.device) if ws is None else ws
    check(lib().salt_iamax(n, _strided(x, n, incx, "x", incx > 0), incx, _dev(result), _dev(ws),
                           ws.numel() * ws.element_size(), d, _stream_ptr(stream)))
    return result


def salt_dot_expr(prog_x, prog_y, operands, scalars, n: int | None = None, result=None, ws=None,
                  stream=None, config=None):
    """Device scalar sum P_i * Q_i for two programs over one operand list,
    in one pass (no vector is written)."""
    d = dtype_code(operands[0])
    for t in operands:
        if dtype_code(t) != d:
            raise TypeError("all operands must share a dtype")
    if n is None:
        n = operands[0].numel()
    result = _result_tensor(d, operands[0].device) if result is None else result
    ws = workspace(n, d, operands[0].device) if ws is None else ws
    px, lx = _prog(prog_x)
    py, ly = _prog(prog_y)
    ops = (ctypes.c_void_p * max(1, len(operands)))(*[_dev(t) for t in operands])
    sc = (ctypes.c_double * max(1, len(scalars)))(*[float(s) for s in scalars])
    args = (px, lx, py, ly, ops, len(operands), sc, len(scalars), n, _dev(result), _dev(ws),
            ws.numel() * ws.element_size(), d, _stream_ptr(stream))
    if config is None:
        check(lib().salt_dot_expr(*args))
    else:
        check(lib().salt_dot_expr_ex(*args, _cfg(config)))
    return result


def salt_nrm2_expr(prog, operands, scalars, n: int | None = None, result=None, ws=None, stream=None,
                   config=None):
    """Device scalar sqrt(sum P_i^2) of a program, in one pass."""
    d = dtype_code(operands[0])
    if n is None:
        n = operands[0].numel()
    result = _result_tensor(d, operands[0].device) if result is None else result
    ws = workspace(n, d, operands[0].device) if ws is None else ws
    p, lp = _prog(prog)
    ops = (ctypes.c_void_p * max(1, len(operands)))(*[_dev(t) for t in operands])
    sc = (ctypes.c_double * max(1, len(scalars)))(*[float(s) for s in scalars])
    args = (p, lp, ops, len(operands), sc, len(scalars), n, _dev(result), _dev(ws),
            ws.numel() * ws.element_size(), d, _stream_ptr(stream))
    if config is None:
        check(lib().salt_nrm2_expr(*args))
    else:
        check(lib().salt_nrm2_expr_ex(*args, _cfg(config)))
    return result


# ---------------------------------------------------------------------------
# host-only helpers
# ---------------------------------------------------------------------------

def salt_program_check(prog: Sequence[int], n_operands: int, n_scalars: int):
    """(stack_need, n_loads) of a valid program; raises SaltError otherwise."""
    parr, plen = _prog(prog)
    sn, nl = ctypes.c_int32(), ctypes.c_int32()
    check(lib().salt_program_check(parr, plen, n_operands, n_scalars, ctypes.byref(sn), ctypes.byref(nl)))
    return sn.value, nl.value


def salt_program_route(prog: Sequence[int], n_operands: int, n_scalars: int) -> int:
    """Catalogue index of the kernel a program runs on, or -1 (interpreter)."""
    parr, plen = _prog(prog)
    r = ctypes.c_int32()
    check(lib().salt_program_route(parr, plen, n_operands, n_scalars, ctypes.byref(r)))
    return r.value


def salt_reduce_expr_route(prog_x: Sequence[int], prog_y: Sequence[int] | None, n_operands: int,
                           n_scalars: int, dtype: int = F64) -> int:
    """Reduction-pair catalogue index the expression reduction runs in
    dtype, ROUTE_COMPILED (its run-time compiled kernel), or -1 (the
    interpreter); prog_y None: nrm2."""
    px, lx = _prog(prog_x)
    py, ly = _prog(prog_y) if prog_y is not None else (None, 0)
    r = ctypes.c_int32()
    check(lib().salt_reduce_expr_route(px, lx, py, ly, n_operands, n_scalars, dtype, ctypes.byref(r)))
    return r.value


def salt_jit_compile_reduce(prog_x: Sequence[int], prog_y: Sequence[int] | None, n_operands: int,
                            n_scalars: int, dtype: int) -> None:
    """Compile the pass-1 kernel of dot(prog_x, prog_y) (prog_y None:
    nrm2(prog_x)) for dtype now (blocking)."""
    px, lx = _prog(prog_x)
    py, ly = _prog(prog_y) if prog_y is not None else (None, 0)
    check(lib().salt_jit_compile_reduce(px, lx, py, ly, n_operands, n_scalars, dtype))


def salt_jit_code_reduce(prog_x: Sequence[int], prog_y: Sequence[int] | None, n_operands: int,
                         n_scalars: int, dtype: int) -> bytes:
    """The compiled code object of a reduction pair (b"" if not compiled)."""
    px, lx = _prog(prog_x)
    py, ly = _prog(prog_y) if prog_y is not None else (None, 0)
    size = ctypes.c_size_t()
    check(lib().salt_jit_code_reduce(px, lx, py, ly, n_operands, n_scalars, dtype, None, 0, ctypes.byref(size)))
    buf = ctypes.create_string_buffer(max(1, size.value))
    check(lib().salt_jit_code_reduce(px, lx, py, ly, n_operands, n_scalars, dtype, buf, size.value,
                                     ctypes.byref(size)))
    return buf.raw[:size.value]


JIT_OFF, JIT_EXPLICIT, JIT_AUTO = 0, 1, 2
ROUTE_COMPILED = -3


def salt_jit_set_mode(mode: int) -> None:
    check(lib().salt_jit_set_mode(mode))


def salt_jit_compile(prog: Sequence[int], n_operands: int, n_scalars: int, dtype: int) -> None:
    """Compile a tree outside the catalogue for dtype now (blocking)."""
    arr, n = _prog(prog)
    check(lib().salt_jit_compile(arr, n, n_operands, n_scalars, dtype))


def salt_jit_code(prog: Sequence[int], n_operands: int, n_scalars: int, dtype: int) -> bytes:
    """The compiled code object of a tree (b"" if not compiled)."""
    arr, n = _prog(prog)
    size = ctypes.c_size_t()
    check(lib().salt_jit_code(arr, n, n_operands, n_scalars, dtype, None, 0, ctypes.byref(size)))
    buf = ctypes.create_string_buffer(max(1, size.value))
    check(lib().salt_jit_code(arr, n, n_operands, n_scalars, dtype, buf, size.value, ctypes.byref(size)))
    return buf.raw[:size.value]


def salt_eval_chunking(n_loads: int, n: int, dtype: int) -> tuple[int, int]:
    """(elements per launch, launches) of an element-wise call."""
    c, k = ctypes.c_int64(), ctypes.c_int64()
    check(lib().salt_eval_chunking(n_loads, n, dtype, ctypes.byref(c), ctypes.byref(k)))
    return c.value, k.value


def salt_eval_route(prog: Sequence[int], n_operands: int, n_scalars: int, dtype: int) -> int:
    """Catalogue index, ROUTE_COMPILED, or -1 (interpreter)."""
    arr, n = _prog(prog)
    r = ctypes.c_int32()
    check(lib().salt_eval_route(arr, n, n_operands, n_scalars, dtype, ctypes.byref(r)))
    return r.value


def salt_catalogue() -> list[tuple[str, list[int]]]:
    """[(name, canonical postfix tokens)] of the ahead-of-time trees."""
    L = lib()
    out = []
    for i in range(L.salt_catalogue_count()):
        buf = (ctypes.c_uint32 * MAX_TOKENS)()
        name = ctypes.c_char_p()
        n = L.salt_catalogue_program(i, buf, MAX_TOKENS, ctypes.byref(name))
        out.append((name.value.decode(), list(buf[:n])))
    return out


def salt_tuning_load(path: str | None = None) -> None:
    check(lib().salt_tuning_load(path.encode() if path else None))


def salt_tuning_lookup(kind: int, route: int, dtype: int, n: int) -> tuple[int, int, int]:
    c = LaunchConfig()
    check(lib().salt_tuning_lookup(kind, route, dtype, n, ctypes.byref(c)))
    return c.as_tuple()


def salt_version() -> int:
    return int(lib().salt_version())
