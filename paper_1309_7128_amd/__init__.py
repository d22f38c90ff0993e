"""Interpolated stencil multigrid (ISM) pressure-Poisson solver for MI355X (gfx950).

The solver itself is the HIP library ``libism.so`` behind the C ABI declared in
``include/ism.h``; this package is its thin Python binding (argument marshalling only).
"""
