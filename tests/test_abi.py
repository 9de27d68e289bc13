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


def test_struct_layouts_match_the_header(tmp_path):
    """The Python binding's ctypes structures have the sizes and field offsets
    a C compiler gives the header's structures."""
    import subprocess
    import paper_1507_05086_amd as cc
    structs = {"cc_round_record": cc._RoundRecord, "cc_run_stats": cc._RunStats,
               "cc_batch_config": cc._BatchConfig, "cc_binomial_params": cc._BinomialParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cc.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c = {}
    for line in out:
        if line:
            parts = line.split()
            c[tuple(parts[:-1])] = int(parts[-1])
    for cname, py in structs.items():
        assert c[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert c[(cname, f)] == getattr(py, f).offset, (cname, f)
