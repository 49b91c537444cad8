"""Batched sparse Krylov solvers for AMD Instinct MI355X (gfx950).

The solver itself is a HIP shared library with a C ABI (``include/batchsolve.h``);
``paper_2308_08417_amd.batchsolve`` is its thin Python binding.  Importing this
package loads nothing: the binding loads the library on first use and raises if
it is missing.
"""
__all__ = ["workloads", "batchsolve"]
