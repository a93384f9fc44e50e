"""MI355X (gfx950) one-sided Jacobi hyperbolic SVD.

``paper_1008_1371_amd.hsvd`` is the ctypes binding of ``libhsvd.so`` (the
C ABI declared in ``include/hsvd.h``); every step of the solve runs in the
HIP kernels of that library.  ``paper_1008_1371_amd.workloads`` draws the
seeded synthetic inputs.
"""
