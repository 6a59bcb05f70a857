"""The C ABI library loads (no GPU needed) and exports every entry point
that include/risrt.h declares; the binding knows the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "risrt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:rt_status|const char\*)\s+(rt_[a-z_]+)\s*\(", src, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    assert "rt_trace" in names and "rt_ris_sum" in names and len(names) >= 15


def test_library_exports_every_declared_symbol():
    from paper_2402_13034_amd import risrt
    if not os.path.exists(risrt.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(risrt.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(risrt.ENTRY_POINTS) == _declared()


def test_env_record_layout_matches_header():
    from paper_2402_13034_amd import risrt
    assert ctypes.sizeof(risrt.RtEnvPath) == 64
    assert risrt.ENV_DTYPE.itemsize == 64
    assert ctypes.sizeof(risrt.RtStats) == 8 * 8 + 8 * 4 + 5 * 8 + 3 * 8 + 6 * 8 + 3 * 4 + 4   # padded to 8


def test_last_error_callable_without_device():
    from paper_2402_13034_amd import risrt
    if not os.path.exists(risrt.LIB_PATH):
        pytest.skip("library not built")
    assert isinstance(risrt.lib().rt_last_error(), bytes)
