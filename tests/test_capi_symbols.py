"""The C-ABI library loads and exports every entry point include/pdf.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdf.h")
LIB = os.path.join(ROOT, "paper_1006_0720_amd", "libpdf.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdf_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("pdf_init_mesh", "pdf_seed_particles", "pdf_advance", "pdf_estimate_stats"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libpdf.so not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
