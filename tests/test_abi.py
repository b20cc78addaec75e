"""CPU-side checks of the C ABI boundary: the library loads, exports every
entry point include/paradv.h declares, the ctypes structs match the header's
field lists, and the Python layer refuses to run without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paradv.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pa_status|void|const char\*)\s+(pa_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2403_01004_amd import paradv
    if not os.path.exists(paradv.LIB_PATH):
        from paper_2403_01004_amd import build
        build.build()
    return paradv


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 15
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing
    assert sorted(lib.EXPORTS) == names


def _struct_fields(name):
    txt = open(HEADER).read()
    m = re.search(r"typedef struct \{((?:(?!typedef struct).)*?)\}\s*" + name + ";", txt, re.S)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        if "(*" in decl:
            fields.append(re.search(r"\(\*(\w+)\)", decl).group(1))
            continue
        decl = re.sub(r"^(const\s+)?\w+\s*\*?\s*", "", decl)
        for part in decl.split(","):
            fields.append(re.sub(r"\[.*\]", "", part).strip().lstrip("*"))
    return fields


@pytest.mark.parametrize("cname,pyname", [("pa_desc", "pa_desc"), ("pa_opts", "pa_opts"),
                                          ("pa_stats", "pa_stats")])
def test_struct_layout_matches_header(lib, cname, pyname):
    py = [f[0] for f in getattr(lib, pyname)._fields_]
    assert py == _struct_fields(cname)


def test_no_cpu_fallback(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2403_01004_amd import inputs
    with pytest.raises(RuntimeError):
        lib.Operator(inputs.shell_mesh(4, 4, 8))


def test_missing_library_fails_loudly(tmp_path):
    from paper_2403_01004_amd import paradv
    saved = paradv._lib
    paradv._lib = None
    try:
        with pytest.raises(ImportError):
            paradv.load(str(tmp_path / "nope.so"))
    finally:
        paradv._lib = saved
