"""MI355X matrix-free interior eigensolver for the random-field spin chain
(arXiv 2012.00217): LOBPCG on the spectral fold (H - sigma I)^2 with a
Jacobi-PCG preconditioner, hand-written HIP kernels for gfx950 behind the C ABI
declared in include/mbl.h.

``workloads`` (seeded inputs) imports without the library; the solver API
(``paper_2012_00217_amd.api``) requires the built libmbl.so.
"""

__all__ = ["api", "workloads", "build"]
