"""Speculative segmented sum CSR SpMV for AMD MI355X (gfx950).

The library is the C ABI in ``include/sss.h`` (``libsss.so``); ``sss`` is its
Python binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is not built.
"""
