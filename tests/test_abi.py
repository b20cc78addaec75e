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
                                          ("pa_stats", "pa_stats"),
                                          ("pa_lpc_train_opts", "pa_lpc_train_opts"),
                                          ("pa_lpc_report", "pa_lpc_report")])
def test_struct_layout_matches_header(lib, cname, pyname):
    py = [f[0] for f in getattr(lib, pyname)._fields_]
    assert py == _struct_fields(cname)


def test_header_constants_match_binding(lib):
    txt = open(HEADER).read()
    assert int(re.search(r"#define PA_LPC_NPARAM (\d+)", txt).group(1)) == lib.PA_LPC_NPARAM
    assert int(re.search(r"PA_NKCLASS = (\d+)", txt).group(1)) == lib.PA_NKCLASS
    assert int(re.search(r"#define PA_MAX_LOG (\d+)", txt).group(1)) == lib.PA_MAX_LOG
    assert int(re.search(r"#define PA_PCG_XGROUP (\d+)", txt).group(1)) == lib.PA_PCG_XGROUP
    box = tuple(int(re.search(r"#define PA_BILU0_B%s (\d+)" % a, txt).group(1)) for a in "IJK")
    assert box == lib.PA_BILU0_BOX
    pcs = dict((k, int(v)) for k, v in re.findall(r"PA_PC_(\w+) = (\d+)", txt))
    assert {k.lower(): v for k, v in pcs.items()} == lib.PCS


def test_he_init_layout(lib):
    th = lib.he_init(4300)
    assert th.dtype.name == "float32" and th.size == lib.PA_LPC_NPARAM
    assert not th[3456:3472].any() and not th[10384:10400].any()   # biases
    assert abs(th[:3456].std() - (2.0 / 216) ** 0.5) < 0.01
    assert abs(th[10400:].std() - (2.0 / 432) ** 0.5) < 0.01


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
