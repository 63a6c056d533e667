"""CPU oracle (test infrastructure only).

A plain FP64 C++ restatement of the connectivity-aware multilevel FEM system
(oracle.cpp), loaded through ctypes.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import this package; the HIP library and
its Python binding never do.
"""
from .oracle import Oracle, build_oracle, ORACLE_SO  # noqa: F401
