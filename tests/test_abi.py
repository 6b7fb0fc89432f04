"""The C-ABI library loads and exports every entry point include/qd.h declares.

CPU-only: nothing is called that needs a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2107_03368_amd", "libqd.so")


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(qd_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("qd_knn_bruteforce", "qd_popcount_rows", "qd_last_error"):
        assert required in names


@pytest.mark.parametrize("name", _declared())
def test_library_exports(name):
    if not os.path.exists(LIB):
        from paper_2107_03368_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(LIB)
    assert hasattr(lib, name), f"{name} declared in include/ but not exported by libqd.so"


def test_version_and_error_string_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    assert lib.qd_version() >= 100
    assert isinstance(lib.qd_last_error(), bytes)


def test_argument_errors_are_reported_before_any_device_work():
    # Fake, never-dereferenced pointers: the checks must reject these calls
    # before touching the device (none is present here).
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    f = lib.qd_knn_bruteforce
    P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    f.argtypes = [P, U64, P, U32, U32, P, P, P, P, P]
    a = P(0x10000)
    assert f(a, 100, a, 5, 0, a, a, a, a, None) == -1          # k = 0
    assert b"k=0" in lib.qd_last_error()
    assert f(a, 100, a, 5, 65, a, a, a, a, None) == -1         # k > QD_MAX_K
    assert f(a, 0, a, 5, 10, a, a, a, a, None) == -1           # empty database
    assert f(None, 100, a, 5, 10, a, a, a, a, None) == -1      # null database
    assert f(P(0x10008), 100, a, 5, 10, a, a, a, a, None) == -1  # misaligned rows
    assert f(a, 100, a, 0, 10, a, a, a, a, None) == 0          # nq = 0 is a no-op


def test_query_tile_values_are_checked_before_device_work():
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    f = lib.qd_knn_bruteforce_shaped
    f.argtypes = [P, U64, P, U32, U32, U32, U32, P, P, P, P, P]
    a = P(0x10000)
    for tile in (3, 32, 255, 257):
        assert f(a, 100, a, 5, 10, tile, 0, a, a, a, a, None) == -1
        assert b"query tile" in lib.qd_last_error()
    g = lib.qd_plan_create
    g.argtypes = [P, P, U64, P, U32, U64, U32, U32, U32, P, U32, ctypes.POINTER(P)]
    h = P()
    assert g(None, a, 100, a, 4, 64, 4, 10, 0, None, 24, ctypes.byref(h)) == -1
    assert b"query tile" in lib.qd_last_error() and not h.value


class _Params(ctypes.Structure):  # qd_search_params, as declared in include/qd.h
    _fields_ = [("order", ctypes.c_int), ("d_scores", ctypes.c_void_p), ("n_scored", ctypes.c_uint32),
                ("waves_per_cu", ctypes.c_uint32), ("d_visited", ctypes.c_void_p), ("n_traced", ctypes.c_uint32),
                ("round1_blocks", ctypes.c_uint32), ("round2_blocks", ctypes.c_uint32),
                ("round_growth", ctypes.c_uint32), ("model", ctypes.c_void_p), ("round1_start", ctypes.c_uint32),
                ("query_split", ctypes.c_uint32)]


def test_plan_takes_a_model_for_the_blocked_order_only():
    # a sequential plan (no tree) given a model is refused before any device
    # work; the model handle is never dereferenced
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    g = lib.qd_plan_create
    g.argtypes = [P, P, U64, P, U32, U64, U32, U32, U32, ctypes.POINTER(_Params), U32, ctypes.POINTER(P)]
    a = P(0x10000)
    prm = _Params()
    prm.model = 0x20000
    h = P()
    assert g(None, a, 100, a, 4, 64, 4, 10, 0, ctypes.byref(prm), 0, ctypes.byref(h)) == -4  # QD_ERR_UNSUPPORTED
    assert b"blocked order only" in lib.qd_last_error() and not h.value


def test_query_split_is_checked_before_device_work():
    # a split that is not 0 or a power of two up to 16 is refused by the
    # search and by a plan before the tree handle is dereferenced
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    P, U32 = ctypes.c_void_p, ctypes.c_uint32
    f = lib.qd_knn_tree
    f.argtypes = [P, P, U32, U32, ctypes.POINTER(_Params), P, P, P, P, P, P, P]
    a = P(0x10000)
    for bad in (3, 6, 32):
        prm = _Params()
        prm.query_split = bad
        assert f(a, a, 8, 10, ctypes.byref(prm), a, a, a, a, None, None, None) == -1
        assert b"query_split" in lib.qd_last_error()
    U64 = ctypes.c_uint64
    g = lib.qd_plan_create
    g.argtypes = [P, P, U64, P, U32, U64, U32, U32, U32, ctypes.POINTER(_Params), U32, ctypes.POINTER(P)]
    prm = _Params()
    prm.query_split = 5
    h = P()
    assert g(a, None, 0, a, 4, 64, 4, 10, 0, ctypes.byref(prm), 0, ctypes.byref(h)) == -1
    assert b"query_split" in lib.qd_last_error() and not h.value


def test_object_score_argument_errors_without_device_work():
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    f = lib.qd_object_scores
    P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    f.argtypes = [P, U64, P, U32, P, U64, P, U32, P, P]
    a = P(0x10000)
    assert f(a, 100, a, 0, a, 10, a, 2, a, None) == -1           # n_obj = 0
    assert b"n_obj" in lib.qd_last_error()
    assert f(a, 100, a, 65537, a, 10, a, 2, a, None) == -1       # ids are uint16
    assert f(a, 100, a, 5, a, 10, a, 0, a, None) == 0            # nqo = 0 is a no-op
    assert f(None, 100, a, 5, a, 10, a, 2, a, None) == -1        # null database with rows
    assert f(a, 100, a, 5, a, 10, None, 2, a, None) == -1        # null offsets
    assert f(a, 100, a, 5, P(0x10008), 10, a, 2, a, None) == -1  # misaligned descriptors


def test_score_rows_argument_errors_without_device_work():
    lib = ctypes.CDLL(LIB)
    f = lib.qd_score_rows
    P, U32 = ctypes.c_void_p, ctypes.c_uint32
    f.argtypes = [P, U32, U32, ctypes.c_int, P, P]
    a = P(0x10000)
    assert f(a, 0, 5, 1, a, None) == 0       # nqo = 0 is a no-op
    assert f(a, 3, 0, 1, a, None) == -1      # no objects
    assert f(None, 3, 5, 1, a, None) == -1   # null scores
    assert f(a, 3, 5, 1, None, None) == -1   # null best


def test_planes_argument_errors_without_device_work():
    lib = ctypes.CDLL(LIB)
    P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    b = lib.qd_planes_build
    b.argtypes = [P, U64, P, ctypes.POINTER(P)]
    h = P()
    a = P(0x10000)
    assert b(None, 10, None, ctypes.byref(h)) == -1           # null database
    assert b(a, 0, None, ctypes.byref(h)) == -1               # no rows
    assert b(P(0x10008), 10, None, ctypes.byref(h)) == -1     # misaligned
    assert b(a, 10, None, None) == -1                         # no output handle
    f = lib.qd_knn_planes
    f.argtypes = [P, P, U32, U32, P, P, P, P, P]
    assert f(None, a, 1, 1, a, a, a, a, None) == -1           # no index
    assert lib.qd_planes_free(None) == 0


def test_noalloc_argument_errors_without_device_work():
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    f = lib.qd_knn_bruteforce_noalloc
    P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    f.argtypes = [P, U64, P, U32, U32, P, P, P, P, P]
    a = P(0x10000)
    assert f(a, 100, a, 5, 0, a, a, a, a, None) == -1            # k = 0
    assert f(a, 0, a, 5, 10, a, a, a, a, None) == -1             # empty database
    assert f(a, 100, a, 5, 10, None, a, a, a, None) == -1        # null output
    assert f(P(0x10008), 100, a, 5, 10, a, a, a, a, None) == -1  # misaligned rows
    assert f(a, 100, a, 0, 10, a, a, a, a, None) == 0            # nq = 0 is a no-op
    # the lists of nq * k keys (one per query at the least) exceed the fixed scratch
    assert f(a, 100, a, 65_537, 64, a, a, a, a, None) == -1
    assert b"scratch" in lib.qd_last_error()


def test_abort_flag_stops_synchronous_calls_before_device_work(tmp_path):
    # a set flag stops the tree build before its first step (fake,
    # never-dereferenced pointers: no device is touched), and the tree load
    # after its host checks; a cleared flag lets the same call proceed to its
    # argument checks and device work
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_tree_file import GOOD, tree_file
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    P, U64 = ctypes.c_void_p, ctypes.c_uint64
    flag = ctypes.c_int(1)
    assert lib.qd_set_abort_flag(ctypes.byref(flag)) == 0
    build = lib.qd_tree_build
    build.argtypes = [P, U64, P, P, ctypes.POINTER(P)]
    h = P()
    try:
        assert build(P(0x10000), 100, None, None, ctypes.byref(h)) == -5  # QD_ERR_ABORTED
        assert b"aborted" in lib.qd_last_error()
        assert build(None, 100, None, None, ctypes.byref(h)) == -1      # argument checks come first
        path = tmp_path / "t.qdtree"
        path.write_bytes(tree_file(**GOOD))
        load = lib.qd_tree_load
        load.argtypes = [ctypes.c_char_p, P, ctypes.POINTER(P)]
        assert load(os.fsencode(str(path)), None, ctypes.byref(h)) == -5
        flag.value = 0
        assert load(os.fsencode(str(path)), None, ctypes.byref(h)) not in (-5, -6, -7)
    finally:
        lib.qd_set_abort_flag(None)
