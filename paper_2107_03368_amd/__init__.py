"""qd: exact Weighted Hamming search over 64x64-bit QUICCI descriptors on MI355X.

Thin Python binding over ``libqd.so`` (the C ABI declared in ``include/qd.h``).
It only marshals arguments: tensors in, device pointers and the current HIP
stream out.  Every step of the search runs in the library's HIP kernels.  If
the library is not built, importing this package fails; there is no fallback.

Descriptors are ``torch.int64`` CUDA tensors of shape ``(n, 64)`` holding the
raw bits of ``uint64[64]`` (word r = image row r, bit c = column c).
"""
import ctypes
import os

import torch  # loads the HIP runtime first, so libqd binds to the same one

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

QD_OK = 0
QD_MAX_K = 64
PAD_IDX = 0xFFFFFFFF

_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32


def _sig(name, args):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = ctypes.c_int
    return f


_lib.qd_last_error.restype = ctypes.c_char_p
_lib.qd_last_error.argtypes = []
_sig("qd_version", [])
_sig("qd_profile_enable", [ctypes.c_int])
_sig("qd_profile_read", [ctypes.c_char_p, _P, _P])
_sig("qd_popcount_rows", [_P, _U64, _P, _P])
_sig("qd_knn_bruteforce", [_P, _U64, _P, _U32, _U32, _P, _P, _P, _P, _P])
_sig("qd_knn_bruteforce_shaped", [_P, _U64, _P, _U32, _U32, _U32, _U32, _P, _P, _P, _P, _P])


class QDError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.qd_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def _check(code, where):
    if code != QD_OK:
        raise QDError(code, where)


def lib():
    """The loaded ctypes library (for ABI-level tests)."""
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _desc(t, name):
    if not (t.is_cuda and t.dtype == torch.int64 and t.dim() == 2 and t.shape[1] == 64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous cuda int64 tensor of shape (n, 64)")
    return t


def _results(nq, k, device):
    return (torch.empty((nq, k), dtype=torch.int32, device=device),
            torch.empty((nq, k), dtype=torch.int32, device=device),
            torch.empty((nq, k), dtype=torch.int32, device=device),
            torch.empty((nq, k), dtype=torch.float32, device=device))


def popcount_rows(db):
    """|t| for every row, as int16 tensor (values 0..4096)."""
    _desc(db, "db")
    out = torch.empty(db.shape[0], dtype=torch.int16, device=db.device)
    _check(_lib.qd_popcount_rows(_ptr(db), db.shape[0], _ptr(out), _stream()), "qd_popcount_rows")
    return out


def knn_bruteforce(db, q, k, query_tile=0, row_parts=0):
    """Exact k-NN by sequential search.  Returns (idx, missed, extra, dist),
    each (nq, k); idx holds uint32 row numbers in int32 storage (PAD_IDX = -1)."""
    _desc(db, "db")
    _desc(q, "q")
    idx, missed, extra, dist = _results(q.shape[0], k, db.device)
    if query_tile or row_parts:
        rc = _lib.qd_knn_bruteforce_shaped(_ptr(db), db.shape[0], _ptr(q), q.shape[0], k, query_tile, row_parts,
                                           _ptr(idx), _ptr(missed), _ptr(extra), _ptr(dist), _stream())
    else:
        rc = _lib.qd_knn_bruteforce(_ptr(db), db.shape[0], _ptr(q), q.shape[0], k, _ptr(idx), _ptr(missed),
                                    _ptr(extra), _ptr(dist), _stream())
    _check(rc, "qd_knn_bruteforce")
    return idx, missed, extra, dist


def profile_enable(on=True):
    _check(_lib.qd_profile_enable(1 if on else 0), "qd_profile_enable")


def profile_read(kernel):
    """(total ms, launches) of a timed kernel since profiling was enabled."""
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    _check(_lib.qd_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)), "qd_profile_read")
    return ms.value, n.value
