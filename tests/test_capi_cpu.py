"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every entry point include/pmh.h declares, the binding declares the
same set, and argument errors are reported before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pmh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmh_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1911_00675_amd import pmh
    if not os.path.exists(pmh.LIB_PATH):
        from paper_1911_00675_amd import build
        build.build()
    return pmh.lib()


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("pmh_init", "pmh_hash_sets", "pmh_estimate", "pmh_destroy", "pmh_server_create"):
        assert n in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    from paper_1911_00675_amd import pmh
    assert sorted(pmh.SIGNATURES) == declared_functions()


def test_status_strings(lib):
    for code in range(0, 12):
        assert lib.pmh_status_str(code)
    assert lib.pmh_status_str(999) == b"unknown status"


def test_argument_errors_without_device(lib):
    out = ctypes.c_void_p()
    assert lib.pmh_init(1, 0, 1, ctypes.byref(out)) == 2        # m = 0
    assert lib.pmh_init(1, 16385, 1, ctypes.byref(out)) == 2    # m too large
    assert lib.pmh_init(1, 1, 3, ctypes.byref(out)) == 3        # m = 1 with PMH3
    assert lib.pmh_init(1, 8, 5, ctypes.byref(out)) == 1        # bad variant
    assert lib.pmh_hash_sets(None, None, None, None, 1, None, None, None, None, None) == 1
    assert lib.pmh_pminhash_sets(None, None, None, None, 1, None, None, None, None, None) == 1
    assert lib.pmh_hash_sets_binary(None, None, None, 1, None, None, None, None, None) == 1
    assert lib.pmh_update_sets(None, None, None, None, 1, None, None, None, None, None, None) == 1
    assert lib.pmh_bbit_pack(None, 1, 8, 1, None, None) == 1
    assert lib.pmh_bbit_allpairs(None, 1, 8, 1, None, None) == 1
    assert lib.pmh_estimate(None, None, None, None, 4, None) == 1


def test_host_estimate(lib):
    import numpy as np
    from paper_1911_00675_amd import pmh
    a = np.array([1, 2, 3, 4], dtype=np.uint64)
    b = np.array([1, 9, 3, 4], dtype=np.uint64)
    ia = np.array([0, 1, 2, 0xFFFFFFFF], dtype=np.uint32)
    ib = np.array([5, 1, 2, 3], dtype=np.uint32)
    assert pmh.estimate(a, ia, b, ib) == 0.5   # component 3 is empty in A
