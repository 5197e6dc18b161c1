"""SALT on MI355X: fused element-wise vector expressions, axpy, dot and nrm2
as hand-written gfx950 HIP kernels behind a C ABI (``libsalt.so``).

Importing the package loads nothing native; :mod:`.salt` loads the library
on first use and raises if it is missing.
"""
__all__ = ["salt", "expr", "batch", "serve", "autotune", "workloads"]
