"""The C-ABI library loads and exports every function include/vns.h declares (CPU only: no compute calls)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "vns.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vns_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("vns_create", "vns_eval_neighbourhood", "vns_run", "vns_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1704_05132_amd import vns
    L = vns.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def test_binding_covers_the_header():
    from paper_1704_05132_amd import vns
    assert sorted(vns.SIGNATURES) == declared_functions()


def test_record_layout_matches_header():
    from paper_1704_05132_amd import vns
    assert vns.RECORD_DTYPE.itemsize == 40
    assert ctypes.sizeof(vns.VNSStats) == 120


def test_create_error_path_without_device_work():
    """Argument validation happens before any device call: a bad size fails with VNS_EINVAL."""
    from paper_1704_05132_amd import vns
    L = vns.lib()
    h = ctypes.c_void_p()
    assert L.vns_create(0, 5, None, None, None, None, None, None, 1, ctypes.byref(h)) == vns.VNS_EINVAL
    assert h.value is None
    assert b"K" in L.vns_last_error(None) or b"NULL" in L.vns_last_error(None)
    assert L.vns_create(3, 200, None, None, None, None, None, None, 1, ctypes.byref(h)) == vns.VNS_EINVAL
