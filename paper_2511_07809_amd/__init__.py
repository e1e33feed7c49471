"""MI355X (gfx950) online tensor-LDA hot path.

The compute lives in libtlda.so (C ABI, include/tlda.h), built in-tree by
``paper_2511_07809_amd.build``; ``paper_2511_07809_amd.tlda`` is its ctypes
binding.  The binding is not imported here so that the package imports on
machines where the library has not been built yet.
"""
__all__ = ["build", "tlda"]
