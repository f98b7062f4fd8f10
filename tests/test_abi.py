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


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and field offsets
    (compiled with the host C compiler against include/labpsd.h)."""
    import shutil
    import subprocess

    import pytest

    import paper_1308_2445_amd as lp
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"labpsd_solve_params": lp.SolveParams, "labpsd_stats": lp.Stats,
               "labpsd_factor_info": lp.FactorInfo}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "labpsd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
