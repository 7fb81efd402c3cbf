"""The C-ABI library loads and exports every entry point declared in
include/powerlu.h (no compute calls: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "powerlu.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(plu_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_2002_07138_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_2002_07138_amd import build as b
        b.build()
    return ctypes.CDLL(pkg.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["plu_create", "plu_destroy", "plu_fixed_rank", "plu_fixed_precision",
                 "plu_residual", "plu_gaussian", "plu_pass", "plu_getrf", "plu_thin_qr",
                 "plu_range_basis", "plu_rank_rule", "plu_status_string"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2002_07138_amd as pkg
    assert sorted(pkg._ENTRY_POINTS) == sorted(set(pkg._ENTRY_POINTS) & set(_declared()))
    assert set(_declared()) <= set(pkg._ENTRY_POINTS)


def test_status_strings_without_gpu(lib):
    lib.plu_status_string.restype = ctypes.c_char_p
    assert lib.plu_status_string(0) == b"ok"
    assert b"tolerance" in lib.plu_status_string(2)
    assert lib.plu_status_string(-3) == b"invalid argument"


def test_oracle_is_not_imported_by_the_product():
    """The product path (package + C sources) never imports or links the oracle."""
    pkg_dir = os.path.join(ROOT, "paper_2002_07138_amd")
    for dirpath, _, files in os.walk(pkg_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "oracle/" not in txt, f


def test_request_and_info_layout_match_the_header(tmp_path):
    """The binding's ctypes mirrors of plu_request / plu_info have the C
    layout (compiled with the system C compiler against include/powerlu.h)."""
    import ctypes
    import shutil
    import subprocess
    import paper_2002_07138_amd as plu
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "lay.c"
    fields = [f for f, _ in plu.PluRequest._fields_]
    body = "".join(f'printf("%zu ", offsetof(plu_request, {f}));' for f in fields)
    ifields = [f for f, _ in plu.PluInfo._fields_]
    body += "".join(f'printf("%zu ", offsetof(plu_info, {f}));' for f in ifields)
    rfields = [f for f, _ in plu.PluResult._fields_]
    body += "".join(f'printf("%zu ", offsetof(plu_result, {f}));' for f in rfields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "powerlu.h"\n'
                   'int main(void){' + body + 'printf("%zu %zu %zu", sizeof(plu_request), '
                   'sizeof(plu_info), sizeof(plu_result));return 0;}\n')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [getattr(plu.PluRequest, f).offset for f in fields]
    want += [getattr(plu.PluInfo, f).offset for f in ifields]
    want += [getattr(plu.PluResult, f).offset for f in rfields]
    want += [ctypes.sizeof(plu.PluRequest), ctypes.sizeof(plu.PluInfo), ctypes.sizeof(plu.PluResult)]
    assert got == want
