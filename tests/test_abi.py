"""The C-ABI library loads and exports every symbol its header declares (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "labpsd.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(labpsd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_header_symbols():
    import paper_1308_2445_amd as lp
    lib = ctypes.CDLL(lp.LIB_PATH)
    names = header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps exactly the header's entry points
    assert sorted(lp.EXPORTED) == names


def test_version_and_error_without_gpu_calls():
    import paper_1308_2445_amd as lp
    assert "labpsd" in lp.version()
    assert isinstance(lp._lib.labpsd_last_error(), bytes)
