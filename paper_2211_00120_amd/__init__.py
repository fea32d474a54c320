"""MI355X-native left-balanced k-d tree construction (arXiv 2211.00120).

The build runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/kdt.h``; ``paper_2211_00120_amd.kdt`` is a thin ctypes binding over
that library.  Importing this package loads nothing; the library is opened on
first use of the binding.
"""
