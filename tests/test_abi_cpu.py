"""CPU checks of the C ABI: the library loads and exports every declared
entry point; the binding names match the header. No compute calls."""
import ctypes
import os
import re

import pytest

from paper_2603_29332_amd import ms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ms.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("ms_model_create", "ms_step_batch", "ms_rollout"):
        assert f in names
    assert sorted(ms.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(ms.LIB_PATH):
        pytest.skip("libms.so not built")
    lib = ctypes.CDLL(ms.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
