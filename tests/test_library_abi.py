"""CPU-side checks of the C ABI: the library loads and exports every entry
point declared in include/libmwalk.h; argument validation that needs no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libmwalk.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\**\s*([a-z_][a-z_0-9]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for want in ("mw_transition", "mw_transition_batch", "frw_extract", "mw_structure_create",
                 "mw_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_2507_09730_amd as mw
    lib = ctypes.CDLL(mw.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2507_09730_amd as mw
    for n in _declared():
        assert hasattr(mw, n), n


def test_validation_without_gpu():
    """Shape checks run before any device work: invalid lattice sizes fail
    with MW_EINVAL and a message."""
    import paper_2507_09730_amd as mw
    lib = ctypes.CDLL(mw.LIB_PATH)
    lib.mw_last_error.restype = ctypes.c_char_p
    dummy = ctypes.c_void_p(16)
    rc = lib.mw_transition(dummy, ctypes.c_int32(7), ctypes.c_int32(0), ctypes.c_uint64(10),
                           ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint32(0), dummy, None,
                           None)
    assert rc == mw.MW_EINVAL
    assert b"even" in lib.mw_last_error()
    rc = lib.mw_transition(dummy, ctypes.c_int32(8), ctypes.c_int32(1), ctypes.c_uint64(10),
                           ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint32(0), dummy, None,
                           None)
    assert rc == mw.MW_EINVAL
    rc = lib.mw_transition(dummy, ctypes.c_int32(66), ctypes.c_int32(0), ctypes.c_uint64(10),
                           ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint32(0), dummy, None,
                           None)
    assert rc == mw.MW_EINVAL
