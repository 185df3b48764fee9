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


def _create(L, vns, K, T, D=None, R=None, kM=None, kR=None, hM=None, hR=None):
    import numpy as np
    z = lambda n, v=1: np.full(n, v, np.int32)
    D = z(K * T) if D is None else np.ascontiguousarray(D, np.int32)
    R = z(K * T, 0) if R is None else np.ascontiguousarray(R, np.int32)
    kM = z(K, 100) if kM is None else np.ascontiguousarray(kM, np.int32)
    kR = z(K, 100) if kR is None else np.ascontiguousarray(kR, np.int32)
    hM = z(K, 2) if hM is None else np.ascontiguousarray(hM, np.int32)
    hR = z(K, 1) if hR is None else np.ascontiguousarray(hR, np.int32)
    h = ctypes.c_void_p()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    st = L.vns_create(K, T, p(D), p(R), p(kM), p(kR), p(hM), p(hR), 1, ctypes.byref(h))
    return st, h


def test_create_status_codes_before_device_work():
    """Every create-time check runs on the host before any HIP call (Section 2 data, the exact-cost bounds):
    EINVAL for sizes, NULL arrays and negative inputs; ERANGE when the int64 cost or the decode's int32
    accumulators could overflow.  No context is returned on error."""
    import numpy as np
    from paper_1704_05132_amd import vns
    L = vns.lib()
    cases = []
    cases.append(("T=0", vns.VNS_EINVAL, dict(K=2, T=0)))
    cases.append(("T>max", vns.VNS_EINVAL, dict(K=2, T=vns.T_MAX + 1)))
    cases.append(("K>max", vns.VNS_EINVAL, dict(K=(1 << 20) + 1, T=1)))
    cases.append(("negative demand", vns.VNS_EINVAL, dict(K=1, T=4, D=[1, -1, 1, 1])))
    cases.append(("negative returns", vns.VNS_EINVAL, dict(K=1, T=4, R=[0, 0, -2, 0])))
    cases.append(("negative setup cost", vns.VNS_EINVAL, dict(K=2, T=3, kM=[5, -5])))
    cases.append(("negative holding cost", vns.VNS_EINVAL, dict(K=2, T=3, hR=[0, -1])))
    cases.append(("demand >= 2^24", vns.VNS_ERANGE, dict(K=1, T=2, D=[1 << 24, 0])))
    cases.append(("returns >= 2^24", vns.VNS_ERANGE, dict(K=1, T=2, R=[0, 1 << 24])))
    # sum D * T >= 2^31 with every demand below 2^24: 128 periods of 2^24 - 1
    cases.append(("sum D * T >= 2^31", vns.VNS_ERANGE, dict(K=1, T=128, D=[(1 << 24) - 1] * 128)))
    # a product's worst-case cost >= 2^47: T (kM + kR) alone with kM = kR = 2^31 - 1 and T = 128
    cases.append(("cost bound >= 2^47", vns.VNS_ERANGE,
                  dict(K=1, T=128, kM=[2 ** 31 - 1], kR=[2 ** 31 - 1], hM=[2 ** 31 - 1], D=[200] * 128)))
    for what, want, kw in cases:
        K, T = kw.pop("K"), kw.pop("T")
        if K > 1 << 20:   # rejected on K alone: no arrays of that size are needed
            h = ctypes.c_void_p()
            one = np.ones(1, np.int32).ctypes.data_as(ctypes.c_void_p)
            st = L.vns_create(K, 1, one, one, one, one, one, one, 1, ctypes.byref(h))
        else:
            st, h = _create(L, vns, K, T, **kw)
        assert st == want, (what, st, L.vns_last_error(None))
        assert h.value is None, what
        assert L.vns_last_error(None), what


def test_null_context_and_argument_status_codes():
    """Calls on a NULL context or with NULL required outputs return VNS_EINVAL without touching a device."""
    from paper_1704_05132_amd import vns
    L = vns.lib()
    v = ctypes.c_int64()
    n = ctypes.c_size_t()
    assert L.vns_run(None, 1) == vns.VNS_EINVAL
    assert L.vns_eval_neighbourhood(None, 7, 0, None, None, None, None, None) == vns.VNS_EINVAL
    assert L.vns_get_option(None, 1, ctypes.byref(v)) == vns.VNS_EINVAL
    assert L.vns_workspace_bytes(None, 1, ctypes.byref(n)) == vns.VNS_EINVAL
    assert L.vns_bind_workspace(None, None, 0, 0) == vns.VNS_EINVAL
    assert L.vns_get_solution(None, 0, 0, None, None) == vns.VNS_EINVAL
    assert L.vns_num_chains(None) == 0
    L.vns_destroy(None)   # accepted


def test_failure_injection_arguments():
    """The test hook rejects unknown kinds and negative countdowns, and 0 clears an injection."""
    from paper_1704_05132_amd import vns
    L = vns.lib()
    assert L.vns_test_inject_failure(3, 1) == vns.VNS_EINVAL
    assert L.vns_test_inject_failure(vns.INJECT_ALLOC, -1) == vns.VNS_EINVAL
    assert L.vns_test_inject_failure(vns.INJECT_ALLOC, 0) == vns.VNS_OK
    assert L.vns_test_inject_failure(vns.INJECT_DEVICE, 0) == vns.VNS_OK
