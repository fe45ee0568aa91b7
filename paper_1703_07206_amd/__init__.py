"""MI355X-native single-grid multi-level (SGML) elliptic solver.

The solver itself lives in the HIP library ``libsgml.so`` (C-ABI declared in
``include/sgml.h``); ``paper_1703_07206_amd.sgml`` is its thin ctypes
binding.  Importing this package loads nothing: the library is opened on the
first solver call, and that call raises if the library is missing.
"""
__all__ = ["sgml", "workloads"]
