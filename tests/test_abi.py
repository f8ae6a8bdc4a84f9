"""The C-ABI library loads on the CPU and exports every symbol include/mx.h
declares (no compute call: there is no GPU here)."""
import os
import re

import pytest

import paper_2311_05322_amd as mx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mx_[a-z_0-9]+)\s*\(", src)))


def test_header_matches_binding():
    assert declared_functions() == sorted(mx.EXPORTS)


@pytest.mark.skipif(not os.path.exists(mx.LIB_PATH), reason="libmx.so not built")
def test_library_exports_every_declared_symbol():
    L = mx.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
