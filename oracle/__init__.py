"""FP64 CPU oracle of the SGML method -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.

* ``oracle.core``  -- ctypes binding of ``sgml_oracle.c`` (the literal,
  full-grid implementation of Algorithms 1-3 and the residual recurrence).
* ``oracle.exact`` -- exact discrete solutions from textbook/library
  routines (DST/DCT diagonalisation, dense LU, CG) used to pin the oracle.
"""
