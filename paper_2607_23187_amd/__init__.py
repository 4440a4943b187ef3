"""Preconditioned Jacobi eigensolver with gap-aware pivoting on MI355X (gfx950).

The solver itself is the HIP library ``libjacobi.so`` behind the C ABI of
``include/jacobi.h``; ``paper_2607_23187_amd.jacobi`` is a thin ctypes binding over it
that takes torch tensors for device memory and streams.  Importing the package loads
nothing; the library is loaded on first use of ``paper_2607_23187_amd.jacobi``.
"""
