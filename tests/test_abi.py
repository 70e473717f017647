"""The C-ABI library loads and exports every entry point include/ip.h declares
(no compute: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ip.h")
LIB = os.path.join(ROOT, "paper_2406_04795_amd", "libip.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ip_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ip_create", "ip_destroy", "ip_problem_create", "ip_trace", "ip_check",
                 "ip_check_cells", "ip_feval", "ip_cells_download"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libip.so not built"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2406_04795_amd import ip
    assert set(ip.EXPORTED) == set(_declared())
