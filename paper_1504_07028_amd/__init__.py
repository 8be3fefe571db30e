"""MI355X (gfx950) implementation of the SegSALSA-STR SALSA iteration (arXiv 1504.07028).

The solver lives in libsegsalsa.so (HIP kernels behind a C ABI, include/segsalsa.h);
`paper_1504_07028_amd.segsalsa` is its thin ctypes binding.  Importing this package
does not load the library; the first call into the binding does, and fails if the
library has not been built.
"""
__all__ = ["segsalsa"]
