"""Seeded synthetic workloads for QUICCI descriptor search.

Test and benchmark input only: this package draws descriptors, queries and
query objects, and holds no step of the search method.  Both the CPU oracle
and the GPU library consume its arrays.

Descriptor layout: ``uint64[64]`` per descriptor; word r is image row r and
bit c of it is column c (bit index ``b = 64*r + c``).  Arrays are returned as
``numpy.uint64`` of shape ``(n, 64)``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

# Popcount window of a database descriptor: 2% .. 8% of 4096 bits.
MIN_BITS = 82
MAX_BITS = 327
# 0.2% of 4096 bits flipped in every query.
N_FLIP = 8


def build():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO,
                           os.path.join(_HERE, "synth.c"), "-lm"])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        U64 = ctypes.c_uint64
        D = ctypes.c_double
        I = ctypes.c_int
        lib.sy_gen_db.argtypes = [P, U64, U64, U64, I, I]
        lib.sy_gen_queries.argtypes = [P, U64, U64, U64, D, D, I, P, P, P]
        lib.sy_gen_query_objects.argtypes = [U64, U64, U64, U64, U64, U64, P, P, P]
        lib.sy_poisson_arrivals.argtypes = [U64, D, U64, P]
        lib.sy_uniform_f32.argtypes = [P, U64, U64, ctypes.c_float, ctypes.c_float]
        lib.sy_permutation.argtypes = [P, U64, U64]
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def gen_db(n, seed, first=0, out=None):
    """Rows ``first .. first+n-1`` of the database drawn from ``seed``."""
    lib = _load()
    if out is None:
        out = np.empty((n, 64), dtype=np.uint64)
    assert out.shape == (n, 64) and out.dtype == np.uint64 and out.flags.c_contiguous
    lib.sy_gen_db(_ptr(out), first, n, seed, MIN_BITS, MAX_BITS)
    return out


def gen_queries(db, nq, seed, pmin, pmax, nflip=N_FLIP, src=None):
    """Partial noisy copies of database rows.  Returns (queries, source rows)."""
    lib = _load()
    db = np.ascontiguousarray(db, dtype=np.uint64)
    q = np.empty((nq, 64), dtype=np.uint64)
    s = np.empty(nq, dtype=np.uint32)
    src_in = None if src is None else np.ascontiguousarray(src, dtype=np.uint32)
    lib.sy_gen_queries(_ptr(db), db.shape[0], nq, seed, pmin, pmax, nflip, _ptr(src_in), _ptr(q), _ptr(s))
    return q, s


def gen_query_objects(n_obj, per_obj, nqo, seed, mmin, mmax):
    """Source rows of ``nqo`` query objects, as CSR ``(offsets[nqo+1], rows, obj)``.

    Each query object takes between mmin and mmax distinct rows of one random
    database object, in random order (the order in which its descriptors are
    later submitted)."""
    lib = _load()
    off = np.zeros(nqo + 1, dtype=np.uint64)
    lib.sy_gen_query_objects(n_obj, per_obj, nqo, seed, mmin, mmax, _ptr(off), None, None)
    off = np.cumsum(off).astype(np.uint64)
    rows = np.empty(int(off[-1]), dtype=np.uint32)
    obj = np.empty(nqo, dtype=np.int32)
    lib.sy_gen_query_objects(n_obj, per_obj, nqo, seed, mmin, mmax, _ptr(off), _ptr(rows), _ptr(obj))
    return off, rows, obj


def poisson_arrivals(n, rate, seed):
    lib = _load()
    t = np.empty(n, dtype=np.float64)
    lib.sy_poisson_arrivals(n, rate, seed, _ptr(t))
    return t


def uniform_f32(n, seed, lo, hi):
    lib = _load()
    out = np.empty(n, dtype=np.float32)
    lib.sy_uniform_f32(_ptr(out), n, seed, lo, hi)
    return out


def permutation(n, seed):
    lib = _load()
    out = np.empty(n, dtype=np.uint32)
    lib.sy_permutation(_ptr(out), n, seed)
    return out


def from_bits(nrows, bit_lists):
    """Descriptors from explicit lists of set bit indices (b = 64*row + col)."""
    out = np.zeros((nrows, 64), dtype=np.uint64)
    for i, bits in enumerate(bit_lists):
        for b in bits:
            out[i, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return out
