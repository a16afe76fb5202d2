"""MI355X (gfx950) particle hot path of the stand-alone PDF method for
turbulent flows on unstructured triangle grids (Bakosi 2008).

The computation lives in libpdf.so (HIP kernels behind the C ABI of
include/pdf.h); this package is its Python binding.  Importing `Context`
loads the library and raises if it has not been built.
"""
from __future__ import annotations

__all__ = ["Context", "PdfError", "workload_context"]


def __getattr__(name):
    if name in ("Context", "PdfError"):
        from . import _lib
        return getattr(_lib, name)
    if name == "workload_context":
        from .runner import workload_context
        return workload_context
    raise AttributeError(name)
