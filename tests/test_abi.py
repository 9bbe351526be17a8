"""The C-ABI library loads and exports every entry point the header declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

import paper_2206_05843_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sptrsv.h")).read()
    return sorted(set(re.findall(r"\b(sptrsv_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(pkg.EXPORTS)


def test_library_exports_all_symbols():
    lib = ctypes.CDLL(pkg.sptrsv.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_names():
    lib = pkg.lib()
    for i, nm in enumerate(pkg.sptrsv.STATUS_NAMES):
        assert lib.sptrsv_status_name(i).decode() == "SPTRSV_" + ("OK" if nm == "OK" else "ERR_" + nm)
