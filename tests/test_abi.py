"""The C-ABI library loads and exports every symbol the header declares
(no GPU work: only symbol lookup and host-side error strings)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cmm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(cmm_\w+)\s*\(", src, re.M)))


def test_header_declares_the_binding_names():
    import paper_1108_1320_amd as pkg
    assert set(_declared()) == set(pkg.EXPORTED)


def test_library_exports_every_symbol():
    import paper_1108_1320_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libcmm.so not built")
    lib = ctypes.CDLL(pkg.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_strerror_and_null_arguments():
    import paper_1108_1320_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libcmm.so not built")
    lib = pkg.load()
    assert lib.cmm_strerror(0) == b"ok"
    assert lib.cmm_strerror(-1) == b"invalid argument"
    assert lib.cmm_ctx_create(0, None, None) == pkg.CMM_EINVAL
    assert lib.cmm_sketch_free(None) == pkg.CMM_EINVAL
    assert lib.cmm_ctx_destroy(None) == pkg.CMM_EINVAL
