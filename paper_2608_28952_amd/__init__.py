"""MI355X-native blocked Jacobi eigensolver and one-sided Jacobi SVD.

The compute path is the C-ABI library ``libjacobi.so`` (HIP kernels for
gfx950) declared in ``include/jacobi.h``; ``paper_2608_28952_amd.jacobi`` is
its thin ctypes binding.  Submodules are imported on demand so that the input
generators can be used on hosts without a GPU.
"""
__version__ = "0.1.0"
