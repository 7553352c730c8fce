"""MI355X library for model-predictive minimal-intervention shared control.

The compute path lives in libmpmi.so (HIP for gfx950, C ABI in include/mpmi.h);
``paper_1906_02318_amd.mpmi`` is its Python binding.  Importing this package
does not load the library; the binding loads it on first use and raises if it
has not been built.
"""
__all__ = ["mpmi"]
