"""camfe: connectivity-aware multilevel finite elements (Chuang & Kazhdan,
arXiv 1505.03615) on AMD MI355X.

The compute path is libcamfe.so (HIP kernels for gfx950) behind the C ABI of
include/camfe.h; `camfe` is its Python binding and `meshgen` produces the
seeded synthetic inputs.  Nothing is loaded at import time.
"""
__all__ = ["camfe", "meshgen", "build"]
