"""Host-side checks of the C ABI that need no GPU: every function declared in
include/apex.h is exported by libapex.so; argument validation of the host-only
calls; the id <-> multi-index map against the oracle's."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads.gen as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apex.h")
SO = os.path.join(ROOT, "paper_2510_24380_amd", "libapex.so")

needs_lib = pytest.mark.skipif(not os.path.exists(SO), reason="libapex.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apex_[a-z_0-9]+)\s*\(", text)))


@needs_lib
def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(SO)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@needs_lib
def test_library_validation_and_decode():
    from paper_2510_24380_amd import binding as B
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced by the host-only calls
    ns = np.array([2, 3, 2], np.uint32)
    ss = np.array([3, 4, 2, 3, 5, 7, 6], np.uint32)
    desc = B.LibraryDesc(3, ns.ctypes.data, ss.ctypes.data, 8, fake)
    h = ctypes.c_void_p()
    assert L.apex_library_create(ctypes.byref(desc), ctypes.byref(h)) == 0
    n = ctypes.c_uint64()
    assert L.apex_library_num_compounds(h, ctypes.byref(n)) == 0
    assert n.value == 3 * 4 + 2 * 3 * 5 + 7 * 6
    ids = np.arange(n.value, dtype=np.uint64)
    r = np.zeros(n.value, np.uint32)
    s = np.zeros((n.value, 3), np.uint32)
    assert L.apex_decode_ids(h, ids.ctypes.data, ids.size, r.ctypes.data, s.ctypes.data) == 0
    lib_h = g.Library(ns, ss, 8, np.zeros((int(ss.sum()), 8), np.float32))
    r2, s2 = oracle.decode(lib_h, ids)
    assert np.array_equal(r, r2) and np.array_equal(s, s2)
    bad = np.array([n.value], np.uint64)
    assert L.apex_decode_ids(h, bad.ctypes.data, 1, r.ctypes.data, s.ctypes.data) == -1
    assert b"out of range" in L.apex_last_error()
    L.apex_library_destroy(h)
    # invalid descriptions
    for ns_bad, ss_bad in (([4], [1, 1, 1, 1]), ([2], [3, 0])):
        a = np.array(ns_bad, np.uint32)
        b = np.array(ss_bad, np.uint32)
        d = B.LibraryDesc(1, a.ctypes.data, b.ctypes.data, 8, fake)
        assert L.apex_library_create(ctypes.byref(d), ctypes.byref(h)) == -1
    d = B.LibraryDesc(1, ns.ctypes.data, ss.ctypes.data, 8, None)
    assert L.apex_library_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert L.apex_status_string(-2) == b"APEX_E_NOMEM"


@needs_lib
def test_decoder_validation():
    from paper_2510_24380_amd import binding as B
    L = B.lib()
    ptrs = (ctypes.c_void_p * 3)(0x1000, 0x2000, 0x3000)

    def create(dims, act=2):
        dd = np.array(dims, np.uint32)
        d = B.DecoderDesc(len(dims) - 1, dd.ctypes.data, act, ctypes.cast(ptrs, ctypes.c_void_p),
                          ctypes.cast(ptrs, ctypes.c_void_p))
        h = ctypes.c_void_p()
        st = L.apex_decoder_create(ctypes.byref(d), ctypes.byref(h))
        if st == 0:
            L.apex_decoder_destroy(h)
        return st

    assert create([256, 512, 512, 15]) == 0
    assert create([64, 128, 5], act=1) == 0
    assert create([64, 128, 5], act=7) == -1
    assert create([64, 128, 17]) == -4        # more heads than one MFMA tile
    assert create([64, 100, 5]) == -4         # unsupported hidden width
    assert create([64, 128, 64, 5]) == 0
    assert create([64, 128, 40, 5]) == -4     # second hidden width not a multiple of 32
    assert create([64, 0, 5]) == -1
    assert create([64, 28]) == 0             # the paper's 28-head linear probe
    assert create([64, 32]) == 0
    assert create([64, 33]) == -4            # more than 32 linear heads
    assert create([64, 5]) == 0              # linear probe (one layer)
