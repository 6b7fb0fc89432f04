"""The tree file format, checked on the host: a file written here by hand
from the documented layout passes every check of qd_tree_load, and every
kind of damage is refused with QD_ERR_FORMAT before any device work (no GPU
is needed for that).  Layout: a 64-byte header (magic "QDTREE\\0\\0", version
1, flags, n, n_nodes, max_leaf, reserved, payload bytes, payload hash, header
hash), then rows, perm, child pairs, begin and count, each padded with zeros
to 8 bytes; hashes are FNV-1a over little-endian 64-bit words."""
import ctypes
import os
import struct

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2107_03368_amd", "libqd.so")
QD_ERR_FORMAT, QD_ERR_IO = -6, -7
M64 = (1 << 64) - 1


def fnv(data, h=0xcbf29ce484222325):
    assert len(data) % 8 == 0
    for (w,) in struct.iter_unpack("<Q", data):
        h = ((h ^ w) * 0x100000001b3) & M64
    return h


def pad(b):
    return b + b"\0" * (-len(b) % 8)


def tree_file(rows, perm, child, begin, count, flags=2, max_leaf=2, version=1, payload_edit=None):
    n, nn = len(rows), len(begin)
    payload = (pad(np.asarray(rows, np.uint64).tobytes()) + pad(np.asarray(perm, np.uint32).tobytes())
               + pad(np.asarray(child, np.int32).tobytes()) + pad(np.asarray(begin, np.uint32).tobytes())
               + pad(np.asarray(count, np.uint32).tobytes()))
    if payload_edit:
        payload = payload_edit(payload)
    head = b"QDTREE\0\0" + struct.pack("<IIQQIIQQ", version, flags, n, nn, max_leaf, 0, len(payload), fnv(payload))
    return head + struct.pack("<Q", fnv(head)) + payload


# three rows; the root (rows 0-2) splits into node 1 (leaf-order rows 0-1) and node 2 (row 2)
ROWS = np.arange(3 * 64, dtype=np.uint64).reshape(3, 64) * np.uint64(0x9E3779B97F4A7C15)
GOOD = dict(rows=ROWS, perm=[2, 0, 1], child=[[1, 2], [-1, -1], [-1, -1]], begin=[0, 0, 2], count=[3, 2, 1])


@pytest.fixture(scope="module")
def load():
    lib = ctypes.CDLL(LIB)
    lib.qd_last_error.restype = ctypes.c_char_p
    f = lib.qd_tree_load
    f.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]

    def run(data, tmp_path):
        p = tmp_path / "t.qdtree"
        p.write_bytes(data)
        h = ctypes.c_void_p()
        rc = f(os.fsencode(str(p)), None, ctypes.byref(h))
        return rc, lib.qd_last_error().decode()
    return run


def test_a_file_written_from_the_layout_passes_every_check(load, tmp_path):
    rc, msg = load(tree_file(**GOOD), tmp_path)
    # every host check passes; what follows needs a device (absent here: an
    # allocation or device error), or succeeds where one is present
    assert rc not in (QD_ERR_FORMAT, QD_ERR_IO), msg


def _edit(at, value):
    def f(b):
        b = bytearray(b)
        b[at] ^= value
        return bytes(b)
    return f


@pytest.mark.parametrize("case", [
    "payload byte", "header byte", "magic", "version", "truncated", "longer", "child order", "child range",
    "split", "perm", "padding", "unknown flag", "too many nodes"])
def test_damage_is_refused_as_a_format_error(load, tmp_path, case):
    g = dict(GOOD)
    if case == "payload byte":
        data = tree_file(**g)
        data = data[:64 + 100] + bytes([data[64 + 100] ^ 0x10]) + data[64 + 101:]
    elif case == "header byte":
        data = bytearray(tree_file(**g))
        data[16] ^= 1  # n, without fixing the header hash
        data = bytes(data)
    elif case == "magic":
        data = b"QDTREF" + tree_file(**g)[6:]
    elif case == "version":
        data = tree_file(**g, version=2)
    elif case == "truncated":
        data = tree_file(**g)[:-8]
    elif case == "longer":
        data = tree_file(**g) + b"\0" * 8
    elif case == "child order":
        data = tree_file(**{**g, "child": [[2, 1], [-1, -1], [-1, -1]]})
    elif case == "child range":
        data = tree_file(**{**g, "child": [[1, 2], [3, 4], [-1, -1]]})
    elif case == "split":
        data = tree_file(**{**g, "begin": [0, 0, 1]})
    elif case == "perm":
        data = tree_file(**{**g, "perm": [2, 0, 2]})
    elif case == "padding":
        # perm is 12 bytes: its last 4 padding bytes must be zero (hash kept consistent)
        at = 3 * 512 + 12
        data = tree_file(**g, payload_edit=_edit(at, 1))
    elif case == "unknown flag":
        data = tree_file(**g, flags=6)
    elif case == "too many nodes":
        data = tree_file(**{**g, "child": [[1, 2], [-1, -1], [-1, -1], [-1, -1], [-1, -1]],
                            "begin": [0, 0, 2, 0, 0], "count": [3, 2, 1, 1, 1]})
    rc, msg = load(data, tmp_path)
    assert rc == QD_ERR_FORMAT, (case, rc, msg)


def test_missing_file_is_an_io_error(tmp_path):
    lib = ctypes.CDLL(LIB)
    f = lib.qd_tree_load
    f.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert f(os.fsencode(str(tmp_path / "none")), None, ctypes.byref(h)) == QD_ERR_IO
    assert f(None, None, ctypes.byref(h)) == -1
