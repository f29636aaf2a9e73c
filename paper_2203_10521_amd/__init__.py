"""MI355X (gfx950) outer-volume engine for variational hierarchical OBBs.

The computation lives in libobbv.so (HIP kernels behind the C ABI of
include/obbv.h); ``paper_2203_10521_amd.api`` is its Python binding.  Importing
the package does not load the library; the binding's first call does, and
raises if it is not built.
"""
