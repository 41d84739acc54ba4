"""MI355X (gfx950) D2V16 windowed-FFT thermal liquid-vapour lattice Boltzmann library.

The method (arXiv 1403.3746) runs in hand-written HIP kernels behind the C ABI of
include/lbfft.h; ``lbfft`` is the Python binding and ``workloads`` builds seeded inputs.
"""
