"""rsolve: recycled GMRES(m) for sequences of convection-diffusion systems on AMD Instinct MI355X.

The solver runs in hand-written HIP kernels behind a C-ABI library
(``include/rsolve.h``); ``paper_1807_09467_amd.rsolve`` is its thin ctypes
binding and ``paper_1807_09467_amd.workload`` the seeded input generator.
"""
