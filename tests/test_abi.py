"""The C-ABI library loads and exports every symbol its header declares (no
GPU needed), and the compute entry points reject bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

fd = pytest.importorskip("paper_cs_0404008_amd")


def declared_functions(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(fdot_\w+|fgemv_\w+|fgemm_\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions(os.path.join(ROOT, "include", "fdot.h"))
    assert len(names) >= 20
    lib = ctypes.CDLL(fd.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_synth_device_library_exports():
    lib = ctypes.CDLL(os.path.join(ROOT, "synth", "libsynth.so"))
    assert hasattr(lib, "synth_fill")


def test_bad_arguments_fail_synchronously():
    L = fd.lib()
    null = ctypes.c_void_p(0)
    # null field handle
    assert L.fdot_modp(null, null, null, 0, null, null) == -1
    assert L.fdot_modp_many(null, 1, null, null, null) == -1
    assert L.fgemm_modp(null, 1, 1, 1, null, 1, null, 1, null, 1, null) == -1
    assert L.fgemv_modp(null, 1, 1, null, 1, null, null, null) == -1
    assert L.fdot_field_destroy(null) == -1
    out = ctypes.c_void_p()
    assert L.fdot_field_create(32751, 0, None, ctypes.byref(out)) == -2
    assert L.fdot_field_create(32749, 9, None, ctypes.byref(out)) == -1
    assert L.fdot_field_create(65537, 3, None, ctypes.byref(out)) == -3
    # options checked before any device work: a block above lambda, a
    # schedule the representation lacks, nonzero reserved words
    O = fd.Options
    assert L.fdot_field_create(67108859, 2, ctypes.byref(O(0, 0, 3)), ctypes.byref(out)) == -3
    assert L.fdot_field_create(67108859, 2, ctypes.byref(O(0, 3, 0)), ctypes.byref(out)) == -4
    assert L.fdot_field_create(251, 4, ctypes.byref(O(0, 4, 0)), ctypes.byref(out)) == -4
    assert L.fdot_field_create(32749, 0, ctypes.byref(O(0, 9, 0)), ctypes.byref(out)) == -1
    bad = O(0, 0, 0)
    bad.reserved[1] = 1
    assert L.fdot_field_create(32749, 0, ctypes.byref(bad), ctypes.byref(out)) == -1
    assert L.fdot_validate(null, null, 0, null, null) == -1
    assert L.fdot_tune_set(None, 1) == -1
