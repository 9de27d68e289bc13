"""The C-ABI library loads and exports every function include/cc.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "cc.h")).read()
    return sorted(set(re.findall(r"CC_API\s+[\w\s\*]+?\b(cc_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("cc_graph_from_csr", "cc_c4", "cc_clusterwild", "cc_cost", "cc_set_eps_policy"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1507_05086_amd as cc
    lib = ctypes.CDLL(cc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    for n in cc.ABI_FUNCTIONS:
        assert n in declared_functions()


def test_policy_validation_on_host():
    import numpy as np
    import paper_1507_05086_amd as cc
    import pytest
    with pytest.raises(cc.CCError):
        cc.cc_set_eps_policy(cc.CC_EPS_TRACE, np.array([3, 0], np.int64))
    with pytest.raises(cc.CCError):
        cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, np.zeros(5, np.float32))
    with pytest.raises(cc.CCError):
        cc.cc_set_eps_policy(7)
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
