"""MI355X-native discrete-forcing immersed-boundary fractional-step solver
(arXiv 2402.17337): HIP kernels for gfx950 behind a C ABI, with a thin
ctypes binding.  Import `paper_2402_17337_amd.ibm` for the solver."""
