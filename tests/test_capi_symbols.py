"""The C-ABI library loads on a machine without a GPU and exports every
function include/boostcom.h declares (no compute call is made here)."""
import ctypes
import os
import re

import paper_2407_07308_amd as bc

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "boostcom.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    assert declared() == bc.exported_symbols()


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(bc.LIB_PATH)
    for name in declared():
        assert hasattr(L, name), name


def test_strerror_is_host_only():
    L = bc.lib()
    assert L.bc_strerror(0) == b"ok"
    assert L.bc_strerror(bc.BC_ERR_LEVEL) == b"out of levels or noise budget"
    assert L.bc_ct_words(None, 0, 2) == 0
