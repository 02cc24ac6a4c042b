"""MI355X (gfx950) library for the DFPT Hubbard-response Sternheimer path.

The compute path is the HIP library ``libhp.so`` (sources in ``csrc/``, C ABI
in ``include/hp.h``); ``hp`` is its ctypes binding.  ``build.build()``
compiles the library in-tree with hipcc for gfx950.
"""
__all__ = ["hp", "build"]
