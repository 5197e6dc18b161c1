"""Plant plausible mistakes in copies of the oracle (on the CPU) and check
that the pins of ``test_oracle_pins.py`` catch every one of them.

Each mutant is a one-line textual change of ``oracle/salt_oracle.c``, built
with the oracle's own flags into a temporary directory. The real oracle is
never modified.
"""
from __future__ import annotations

import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

MUTANTS = {
    # a transposed operand in SUB
    "sub_swapped": ("op == OR_SUB ? l - r", "op == OR_SUB ? r - l"),
    # the wrong scalar slot
    "scalar_index": ("st[sp++] = (float)scalars[arg];", "st[sp++] = (float)scalars[0];"),
    # the wrong operand slot in binary64
    "load_index_f64": ("if (op == OR_LOAD) { st[sp++] = ops[arg][i]; continue; }\n            if (op == OR_SCALAR) { st[sp++] = scalars[arg]",
                       "if (op == OR_LOAD) { st[sp++] = ops[0][i]; continue; }\n            if (op == OR_SCALAR) { st[sp++] = scalars[arg]"),
    # a dropped term in Dot2 (the product's rounding error)
    "dot2_drop_product_error": ("s = s + (q + r);", "s = s + q;"),
    # a dropped term in TwoSum
    "twosum_drop_term": ("*e = (a - (*s - z)) + (b - z);", "*e = (a - (*s - z));"),
    # ties rounded up instead of to even (bfloat16)
    "bf16_ties_up": ("if (dropped > 0x8000u || (dropped == 0x8000u && (kept & 1u))) ++kept;",
                     "if (dropped >= 0x8000u) ++kept;"),
    # truncation instead of rounding (binary16 normal range)
    "f16_truncate": ("if (rem > 0x1000u || (rem == 0x1000u && (q & 1u))) ++q; /* carry",
                     "if (0) ++q; /* carry"),
    # an off-by-one exponent in binary16 gradual underflow
    "f16_subnormal_shift": ("int shift = 126 - e;", "int shift = 125 - e;"),
    # a wrong scale of binary16 subnormals on widening
    "f16_widen_subnormal": ("ldexpf((float)m, -24)", "ldexpf((float)m, -25)"),
    # nrm2 without its square root
    "nrm2_no_sqrt": ("*result = sqrt(s);", "*result = s;"),
    # axpy with its operands transposed
    "axpy_transposed": ("y[i] = alpha * x[i] + y[i];", "y[i] = alpha * y[i] + x[i];"),
    # binary32 scalars not rounded to binary32 before use (kept in binary64)
    "f32_axpy_alpha_f64": ("for (int64_t i = 0; i < n; ++i) y[i] = a * x[i] + y[i];",
                           "for (int64_t i = 0; i < n; ++i) y[i] = (float)(alpha * x[i] + y[i]);"),
    # naive loop accumulating in the wrong precision
    "naive_f32_in_f64": ("float s = 0.0f;\n    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];",
                         "double s = 0.0;\n    for (int64_t i = 0; i < n; ++i) s = s + (double)x[i] * y[i];"),
    # the binary64 loop accumulating in binary32
    "naive_f64_in_f32": ("double s = 0.0;\n    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];\n    return s;",
                         "float s = 0.0f;\n    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];\n    return s;"),
    # the binary64 loop dropping the last element
    "naive_f64_drop_last": ("double s = 0.0;\n    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];\n    return s;",
                            "double s = 0.0;\n    for (int64_t i = 0; i + 1 < n; ++i) s = s + x[i] * y[i];\n    return s;"),
    # the binary64 loop with a fused multiply-add
    "naive_f64_fma": ("double s = 0.0;\n    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];\n    return s;",
                      "double s = 0.0;\n    for (int64_t i = 0; i < n; ++i) s = fma(x[i], y[i], s);\n    return s;"),
    # the binary64 loop returning the Dot2 value
    "naive_f64_is_dot2": ("double s = 0.0;\n    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];\n    return s;",
                          "double s = 0.0;\n    oracle_dot2(n, x, y, &s, 0);\n    return s;"),
    # the all-cores loop adding its partials in reverse thread order
    "naive_par_reverse": ("for (int t = 0; t < ran; ++t) s = s + part[t];",
                          "for (int t = ran - 1; t >= 0; --t) s = s + part[t];"),
    # the all-cores loop giving the first threads the remainder
    "naive_par_split": ("hi = (int64_t)((__int128)n * (t + 1) / T);",
                        "hi = t + 1 == T ? n : (int64_t)((__int128)n * (t + 1) / T + (n % T ? 1 : 0));"),
    # negative increments walking forward instead of from the far end
    "blas_negative_forward": ("return inc >= 0 ? i * inc : (n - 1 - i) * (-inc);",
                              "return inc >= 0 ? i * inc : i * (-inc);"),
    # the last element of a negative-increment vector dropped (off by one)
    "blas_negative_off_by_one": ("return inc >= 0 ? i * inc : (n - 1 - i) * (-inc);",
                                 "return inc >= 0 ? i * inc : (n - i) * (-inc) - 1;"),
    # iamax keeping the last of equal magnitudes
    "iamax_last_tie": ("        const double a = fabs(x[i * inc]);\n        if (a > m) {",
                       "        const double a = fabs(x[i * inc]);\n        if (a >= m) {"),
    # iamax on signed values instead of magnitudes (binary32)
    "iamax_signed_f32": ("const float a = fabsf(x[i * inc]);", "const float a = x[i * inc];"),
    # iamax ignoring the increment
    "iamax_unit_stride": ("const double a = fabs(x[i * inc]);", "const double a = fabs(x[i]);"),
    # canonical order: a lane taking 16 consecutive chunks instead of every 256th
    "rc_lane_contiguous": ("(int64_t)j * RC_LANES + l;", "(int64_t)l * RC_CHUNKS + j;"),
    # canonical order: the four lane groups summed sequentially
    "rc_groups_sequential": ("return (g[0] + g[1]) + (g[2] + g[3]);", "return ((g[0] + g[1]) + g[2]) + g[3];"),
    # canonical order: the final tree pairing k with k + h
    "rc_final_tree_pairs": ("for (int k = 0; k < h; ++k) g[k] = g[2 * k] + g[2 * k + 1];",
                            "for (int k = 0; k < h; ++k) g[k] = g[k] + g[k + h];"),
    # canonical order: binary32 compensation without the sum's error
    "rc_drop_sum_error": ("if (kind == 1) cf[p] = cf[p] + (e + fmaf(a, b, -prod));",
                          "if (kind == 1) cf[p] = cf[p] + fmaf(a, b, -prod);"),
    # canonical order: nrm2 without its square root
    "rc_nrm2_no_sqrt": ("if (mode == 1) r = sqrt(r);", "if (mode == 1) r = r;"),
    # canonical order: elements past n read instead of zero (binary64)
    "rc_tail_read": ("double a = i < n ? ((const double *)x)[i] : 0.0, b;",
                     "double a = i < n ? ((const double *)x)[i] : 1.0, b;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "salt_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, "mutation site not found: %s" % name
    mutated = src.replace(old, new)
    c = tmp_path / "mutant.c"
    c.write_text(mutated)
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, str(c), "-o", str(so), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load(str(so)))
    failed = []
    for check_name, check in pins.CHECKS.items():
        try:
            check(oracle)
        except AssertionError:
            failed.append(check_name)
    assert failed, "no pin caught mutant %s" % name
