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
    raise ImportError(f"{LIB_PATH} is not built; build it with python paper_2107_03368_amd/build.py (hipcc for gfx950)")

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


QUERY_TILE_MATRIX = 256  # query_tile: tiles of 16 queries on the matrix cores


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


_sig("qd_knn_bruteforce_noalloc", [_P, _U64, _P, _U32, _U32, _P, _P, _P, _P, _P])
NOALLOC_SCRATCH_BYTES = 32 << 20


def knn_bruteforce_noalloc(db, q, k, out=None):
    """Sequential search that allocates no device memory inside the library
    (its scratch is a fixed array per GPU).  ``out`` = (idx, missed, extra,
    dist) tensors of shape (nq, k) to write into; new ones if omitted."""
    _desc(db, "db")
    _desc(q, "q")
    idx, missed, extra, dist = out if out is not None else _results(q.shape[0], k, db.device)
    for t, dt in zip((idx, missed, extra, dist), (torch.int32, torch.int32, torch.int32, torch.float32)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() >= q.shape[0] * k):
            raise ValueError("outputs must be contiguous cuda tensors of nq x k int32/int32/int32/float32")
    rc = _lib.qd_knn_bruteforce_noalloc(_ptr(db), db.shape[0], _ptr(q), q.shape[0], k, _ptr(idx), _ptr(missed),
                                        _ptr(extra), _ptr(dist), _stream())
    _check(rc, "qd_knn_bruteforce_noalloc")
    return idx, missed, extra, dist


def profile_enable(on=True):
    _check(_lib.qd_profile_enable(1 if on else 0), "qd_profile_enable")


_sig("qd_profile_counter", [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint64)])


def profile_counter(name):
    """A named work counter summed since profiling was enabled."""
    v = ctypes.c_uint64()
    _check(_lib.qd_profile_counter(name.encode(), ctypes.byref(v)), "qd_profile_counter")
    return v.value


def profile_read(kernel):
    """(total ms, launches) of a timed kernel since profiling was enabled."""
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    _check(_lib.qd_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)), "qd_profile_read")
    return ms.value, n.value


# ---------------------------------------------------------------------------
# Dissimilarity Tree
# ---------------------------------------------------------------------------
class _BuildParams(ctypes.Structure):
    _fields_ = [("max_leaf", ctypes.c_uint32), ("store_and_image", ctypes.c_uint32), ("plain_bound", ctypes.c_uint32)]


class _TreeInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("n_nodes", ctypes.c_uint64), ("n_leaves", ctypes.c_uint64),
                ("depth", ctypes.c_uint32), ("max_leaf", ctypes.c_uint32), ("has_and_image", ctypes.c_uint32),
                ("has_pop_range", ctypes.c_uint32)]


class _SearchParams(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("d_scores", ctypes.c_void_p), ("n_scored", ctypes.c_uint32),
                ("waves_per_cu", ctypes.c_uint32), ("d_visited", ctypes.c_void_p), ("n_traced", ctypes.c_uint32),
                ("round1_blocks", ctypes.c_uint32), ("round2_blocks", ctypes.c_uint32),
                ("round_growth", ctypes.c_uint32), ("model", ctypes.c_void_p), ("round1_start", ctypes.c_uint32),
                ("query_split", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("nodes_visited", ctypes.c_uint64), ("leaves_visited", ctypes.c_uint64),
                ("bounds_evaluated", ctypes.c_uint64), ("dists_evaluated", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


ORDER_BEST_FIRST = 0
ORDER_DEPTH_FIRST = 1
ORDER_BLOCKED = 2

_sig("qd_tree_build", [_P, _U64, ctypes.POINTER(_BuildParams), _P, ctypes.POINTER(ctypes.c_void_p)])
_sig("qd_tree_free", [_P])
_sig("qd_tree_info", [_P, ctypes.POINTER(_TreeInfo)])
_sig("qd_tree_export", [_P, _P, _P, _P, _P, _P, _P])
_sig("qd_knn_tree", [_P, _P, _U32, _U32, ctypes.POINTER(_SearchParams), _P, _P, _P, _P, _P,
                     ctypes.POINTER(Stats), _P])


class Tree:
    """A library-owned Dissimilarity Tree (freed with the object)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)
        info = _TreeInfo()
        _check(_lib.qd_tree_info(self._h, ctypes.byref(info)), "qd_tree_info")
        self.n, self.n_nodes, self.n_leaves = info.n, info.n_nodes, info.n_leaves
        self.depth, self.max_leaf, self.has_and_image = info.depth, info.max_leaf, bool(info.has_and_image)
        self.has_pop_range = bool(info.has_pop_range)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None and self._h.value:
            _lib.qd_tree_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def export(self):
        """Host copies: child (n_nodes, 2), begin, count, or_img (n_nodes, 64), [and_img], perm."""
        import numpy as np
        child = np.empty((self.n_nodes, 2), np.int32)
        begin = np.empty(self.n_nodes, np.uint32)
        count = np.empty(self.n_nodes, np.uint32)
        or_img = np.empty((self.n_nodes, 64), np.uint64)
        and_img = np.empty((self.n_nodes, 64), np.uint64) if self.has_and_image else None
        perm = np.empty(self.n, np.uint32)
        p = lambda a: None if a is None else ctypes.c_void_p(a.ctypes.data)
        _check(_lib.qd_tree_export(self._h, p(child), p(begin), p(count), p(or_img), p(and_img), p(perm)),
               "qd_tree_export")
        return dict(child=child, begin=begin, count=count, or_img=or_img, and_img=and_img, perm=perm)


_sig("qd_tree_save", [_P, ctypes.c_char_p])
_sig("qd_tree_load", [ctypes.c_char_p, _P, ctypes.POINTER(ctypes.c_void_p)])


def tree_save(tree, path):
    """Write the tree (rows in leaf order, permutation, structure) to a file."""
    _check(_lib.qd_tree_save(tree.handle, os.fsencode(path)), "qd_tree_save")


def tree_load(path):
    """A tree read from a file written by tree_save, on the current device."""
    h = ctypes.c_void_p()
    _check(_lib.qd_tree_load(os.fsencode(path), _stream(), ctypes.byref(h)), "qd_tree_load")
    return Tree(h.value)


def tree_build(db, max_leaf=32, store_and_image=False, plain_bound=False):
    """plain_bound: the paper's image bound only (no popcount ranges)."""
    _desc(db, "db")
    prm = _BuildParams(max_leaf, 1 if store_and_image else 0, 1 if plain_bound else 0)
    h = ctypes.c_void_p()
    _check(_lib.qd_tree_build(_ptr(db), db.shape[0], ctypes.byref(prm), _stream(), ctypes.byref(h)),
           "qd_tree_build")
    return Tree(h.value)


START_LOWEST_BOUND = 0
START_BOUND_DESCENT = 1


def knn_tree(tree, q, k, order=ORDER_BEST_FIRST, scores=None, query_stats=False, totals=False, waves_per_cu=0,
             schedule=(0, 0, 0), model=None, n_scored=0, start=START_LOWEST_BOUND, split=0):
    """Exact k-NN through the tree.  Returns (idx, missed, extra, dist[, qstats][, totals]).
    schedule: (round-1 blocks, round-2 blocks, growth) of the blocked order, 0 = default.
    split: concurrent subtree searches per query of the per-query orders (0 = default, 1 = none).
    model: a Model that orders the depth-first search (scoring nodes below n_scored,
    0 = default) or picks where the blocked search starts."""
    _desc(q, "q")
    nq = q.shape[0]
    idx, missed, extra, dist = _results(nq, k, q.device)
    qs = torch.empty((nq, 4), dtype=torch.int32, device=q.device) if query_stats else None
    prm = _SearchParams(order, None, n_scored, waves_per_cu, None, 0, *schedule)
    prm.round1_start = start
    prm.query_split = split
    if model is not None:
        prm.model = model.handle.value
    if scores is not None:
        if not (scores.is_cuda and scores.dtype == torch.float32 and scores.dim() == 2 and scores.shape[0] == nq
                and scores.is_contiguous()):
            raise ValueError("scores must be a contiguous cuda float32 tensor (nq, n_scored)")
        prm.d_scores = scores.data_ptr()
        prm.n_scored = scores.shape[1]
    st = Stats()
    _check(_lib.qd_knn_tree(tree.handle, _ptr(q), nq, k, ctypes.byref(prm), _ptr(idx), _ptr(missed), _ptr(extra),
                            _ptr(dist), _ptr(qs), ctypes.byref(st) if totals else None, _stream()), "qd_knn_tree")
    out = [idx, missed, extra, dist]
    if query_stats:
        out.append(qs)
    if totals:
        out.append(st.as_dict())
    return tuple(out)


# ---------------------------------------------------------------------------
# Bit-plane index (small query batches)
_sig("qd_planes_build", [_P, _U64, _P, ctypes.POINTER(ctypes.c_void_p)])
_sig("qd_planes_free", [_P])
_sig("qd_knn_planes", [_P, _P, _U32, _U32, _P, _P, _P, _P, _P])


class Planes:
    """A library-owned bit-plane index of ``db`` (kept alive with it)."""

    def __init__(self, db):
        _desc(db, "db")
        self._db = db  # the index reads the result rows from it
        h = ctypes.c_void_p()
        _check(_lib.qd_planes_build(_ptr(db), db.shape[0], _stream(), ctypes.byref(h)), "qd_planes_build")
        self._h = h
        self.n = db.shape[0]

    def free(self):
        if self._h:
            _lib.qd_planes_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def knn_planes(planes, q, k):
    """Exact k-NN through the bit-plane index: (idx, missed, extra, dist)."""
    _desc(q, "q")
    out = _results(q.shape[0], k, q.device)
    _check(_lib.qd_knn_planes(planes._h, _ptr(q), q.shape[0], k, *(_ptr(t) for t in out), _stream()),
           "qd_knn_planes")
    return out


# ---------------------------------------------------------------------------
# Retrieval by voting
# ---------------------------------------------------------------------------
_sig("qd_retrieve_objects", [_P, _P, _U64, _P, _U32, _P, _U64, _P, _U32, _U32, _U32, ctypes.POINTER(_SearchParams),
                             _P, _P, _P, _P, _P])


def retrieve_objects(qdesc, qoff, obj_of, n_obj, k, threshold=10, tree=None, db=None, order=ORDER_BEST_FIRST,
                     return_nn=False, schedule=(0, 0, 0), model=None, split=0):
    """Vote histogram (nqo, n_obj), winner (nqo,), descriptors used (nqo,)[, neighbour rows].

    qoff: cuda int64 (nqo+1) CSR offsets into qdesc; obj_of: cuda int16 object id per database row.
    model: the tree search's learned order (depth-first and blocked orders)."""
    _desc(qdesc, "qdesc")
    if tree is None:
        _desc(db, "db")
    nqo = qoff.shape[0] - 1
    dev = qdesc.device
    votes = torch.empty((nqo, n_obj), dtype=torch.int32, device=dev)
    winner = torch.empty(nqo, dtype=torch.int32, device=dev)
    used = torch.empty(nqo, dtype=torch.int32, device=dev)
    nn = torch.empty((qdesc.shape[0], k), dtype=torch.int32, device=dev) if return_nn else None
    prm = _SearchParams(order, None, 0, 0, None, 0, *schedule)
    prm.query_split = split
    if model is not None:
        prm.model = model.handle.value
    rc = _lib.qd_retrieve_objects(tree.handle if tree is not None else None, _ptr(db), 0 if db is None else db.shape[0],
                                  _ptr(obj_of), n_obj, _ptr(qdesc), qdesc.shape[0], _ptr(qoff), nqo, k, threshold,
                                  ctypes.byref(prm), _ptr(votes), _ptr(winner), _ptr(used), _ptr(nn), _stream())
    _check(rc, "qd_retrieve_objects")
    return (votes, winner, used, nn) if return_nn else (votes, winner, used)


_sig("qd_retrieve_objects_early", [_P, _P, _U64, _P, _U32, _P, _U64, _P, _U32, _U32, _U32,
                                   ctypes.POINTER(_SearchParams), _P, _P, _P, ctypes.POINTER(ctypes.c_uint64), _P])


def retrieve_objects_early(qdesc, qoff, obj_of, n_obj, k, threshold=10, tree=None, db=None, order=ORDER_BEST_FIRST):
    """Retrieval that stops each query object at the vote threshold.  Returns
    (votes over the descriptors used, winner, used, descriptors searched)."""
    _desc(qdesc, "qdesc")
    if tree is None:
        _desc(db, "db")
    nqo = qoff.shape[0] - 1
    dev = qdesc.device
    votes = torch.empty((nqo, n_obj), dtype=torch.int32, device=dev)
    winner = torch.empty(nqo, dtype=torch.int32, device=dev)
    used = torch.empty(nqo, dtype=torch.int32, device=dev)
    searched = ctypes.c_uint64(0)
    prm = _SearchParams(order, None, 0, 0, None, 0)
    rc = _lib.qd_retrieve_objects_early(tree.handle if tree is not None else None, _ptr(db),
                                        0 if db is None else db.shape[0], _ptr(obj_of), n_obj, _ptr(qdesc),
                                        qdesc.shape[0], _ptr(qoff), nqo, k, threshold, ctypes.byref(prm), _ptr(votes),
                                        _ptr(winner), _ptr(used), ctypes.byref(searched), _stream())
    _check(rc, "qd_retrieve_objects_early")
    return votes, winner, used, searched.value


_sig("qd_object_scores", [_P, _U64, _P, _U32, _P, _U64, _P, _U32, _P, _P])


def object_scores(db, obj_of, n_obj, qdesc, qoff):
    """Summed nearest-neighbour distance of every query object (CSR qoff into
    qdesc) to every database object: cuda float64 (nqo, n_obj)."""
    _desc(db, "db")
    _desc(qdesc, "qdesc")
    nqo = qoff.shape[0] - 1
    scores = torch.empty((nqo, n_obj), dtype=torch.float64, device=qdesc.device)
    rc = _lib.qd_object_scores(_ptr(db), db.shape[0], _ptr(obj_of), n_obj, _ptr(qdesc), qdesc.shape[0], _ptr(qoff),
                               nqo, _ptr(scores), _stream())
    _check(rc, "qd_object_scores")
    return scores


_sig("qd_score_rows", [_P, _U32, _U32, ctypes.c_int, _P, _P])


def score_rows(scores, normalize=True):
    """Best object per query object (int32, -1 if no finite score) and, with
    normalize, the rows of ``scores`` rescaled to [0, 1] in place."""
    if not (scores.is_cuda and scores.dtype == torch.float64 and scores.dim() == 2 and scores.is_contiguous()):
        raise ValueError("scores must be a contiguous cuda float64 tensor of shape (nqo, n_obj)")
    best = torch.empty(scores.shape[0], dtype=torch.int32, device=scores.device)
    rc = _lib.qd_score_rows(_ptr(scores), scores.shape[0], scores.shape[1], 1 if normalize else 0, _ptr(best),
                            _stream())
    _check(rc, "qd_score_rows")
    return best


# ---------------------------------------------------------------------------
# Learned frontier order (MLP)
# ---------------------------------------------------------------------------
MLP_HIDDEN = 256
MLP_FEATURES = 32
MLP_NPARAMS = 1123073

_sig("qd_model_create", [_P, _P, ctypes.POINTER(ctypes.c_void_p)])
_sig("qd_model_free", [_P])
_sig("qd_model_params", [_P, _P, _P])
_sig("qd_model_features", [_P, _P, _P, _P, _U64, _P, _P])
_sig("qd_model_forward", [_P, _P, _U32, _P, _P, _U64, _P, _P])
_sig("qd_model_gradients", [_P, _P, _U32, _P, _P, _P, _P, _U64, _P, _P, _P])
_sig("qd_model_adam_step", [_P, _P, ctypes.c_float, _P])
_sig("qd_model_score_tree", [_P, _P, _P, _U32, _U32, _P, _P])
_sig("qd_trace_pairs", [_P, _U32, _U32, _P, _P, _U32, _P, _P, _P, _U64, _P, ctypes.POINTER(ctypes.c_uint64), _P])
_sig("qd_model_train", [_P, _P, _P, _U32, _U32, _U32, _U32, _U32, ctypes.c_float, _P, _P,
                        ctypes.POINTER(ctypes.c_uint64), _P])


class Model:
    """Library-owned frontier-order model (fp32 masters + bf16 copies)."""

    def __init__(self, params):
        if not (params.is_cuda and params.dtype == torch.float32 and params.numel() == MLP_NPARAMS):
            raise ValueError(f"params must be a cuda float32 tensor of {MLP_NPARAMS} values")
        h = ctypes.c_void_p()
        _check(_lib.qd_model_create(_ptr(params.contiguous()), _stream(), ctypes.byref(h)), "qd_model_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def params(self):
        out = torch.empty(MLP_NPARAMS, dtype=torch.float32, device="cuda")
        _check(_lib.qd_model_params(self._h, _ptr(out), _stream()), "qd_model_params")
        return out

    def free(self):
        if self._h is not None and self._h.value:
            _lib.qd_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _u32(t, name):
    if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous cuda int32 tensor")
    return t


def model_features(tree, q, pair_q, pair_node):
    _desc(q, "q")
    _u32(pair_q, "pair_q")
    _u32(pair_node, "pair_node")
    feat = torch.empty((pair_q.shape[0], MLP_FEATURES), dtype=torch.float32, device=q.device)
    _check(_lib.qd_model_features(tree.handle, _ptr(q), _ptr(pair_q), _ptr(pair_node), pair_q.shape[0], _ptr(feat),
                                  _stream()), "qd_model_features")
    return feat


def model_forward(model, q, pair_q, feat):
    _desc(q, "q")
    _u32(pair_q, "pair_q")
    s = torch.empty(pair_q.shape[0], dtype=torch.float32, device=q.device)
    _check(_lib.qd_model_forward(model.handle, _ptr(q), q.shape[0], _ptr(pair_q), _ptr(feat.contiguous()),
                                 pair_q.shape[0], _ptr(s), _stream()), "qd_model_forward")
    return s


def model_gradients(model, q, qoff, pair_q, feat, labels):
    """(gradient vector, mean loss); pairs grouped by query as qoff (int64, nq+1) says."""
    _desc(q, "q")
    _u32(pair_q, "pair_q")
    g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=q.device)
    loss = torch.empty(1, dtype=torch.float32, device=q.device)
    _check(_lib.qd_model_gradients(model.handle, _ptr(q), q.shape[0], _ptr(qoff), _ptr(pair_q),
                                   _ptr(feat.contiguous()), _ptr(labels.contiguous()), pair_q.shape[0], _ptr(g),
                                   _ptr(loss), _stream()), "qd_model_gradients")
    return g, loss


def model_adam_step(model, grads, lr):
    _check(_lib.qd_model_adam_step(model.handle, _ptr(grads), lr, _stream()), "qd_model_adam_step")


def model_score_tree(model, tree, q, n_scored):
    _desc(q, "q")
    s = torch.empty((q.shape[0], n_scored), dtype=torch.float32, device=q.device)
    _check(_lib.qd_model_score_tree(model.handle, tree.handle, _ptr(q), q.shape[0], n_scored, _ptr(s), _stream()),
           "qd_model_score_tree")
    return s


def knn_tree_traced(tree, q, k, n_traced):
    """Best-first search that also returns the visited bitmap (nq, ceil(n_traced/32)) int32."""
    _desc(q, "q")
    nq = q.shape[0]
    idx, missed, extra, dist = _results(nq, k, q.device)
    vis = torch.empty((nq, (n_traced + 31) // 32), dtype=torch.int32, device=q.device)
    prm = _SearchParams(ORDER_BEST_FIRST, None, 0, 0, vis.data_ptr(), n_traced)
    _check(_lib.qd_knn_tree(tree.handle, _ptr(q), nq, k, ctypes.byref(prm), _ptr(idx), _ptr(missed), _ptr(extra),
                            _ptr(dist), None, None, _stream()), "qd_knn_tree")
    return idx, missed, extra, dist, vis


def trace_pairs(tree, result_idx, visited, n_traced):
    """(pair_q, pair_node, labels, qoff) from a traced search."""
    nq, k = result_idx.shape
    qoff = torch.empty(nq + 1, dtype=torch.int64, device=result_idx.device)
    n = ctypes.c_uint64()
    _check(_lib.qd_trace_pairs(tree.handle, nq, k, _ptr(result_idx), _ptr(visited), n_traced, None, None, None, 0,
                               _ptr(qoff), ctypes.byref(n), _stream()), "qd_trace_pairs")
    npairs = n.value
    pq = torch.empty(npairs, dtype=torch.int32, device=result_idx.device)
    pn = torch.empty(npairs, dtype=torch.int32, device=result_idx.device)
    lab = torch.empty(npairs, dtype=torch.float32, device=result_idx.device)
    _check(_lib.qd_trace_pairs(tree.handle, nq, k, _ptr(result_idx), _ptr(visited), n_traced, _ptr(pq), _ptr(pn),
                               _ptr(lab), npairs, _ptr(qoff), ctypes.byref(n), _stream()), "qd_trace_pairs")
    return pq, pn, lab, qoff


def model_train(model, tree, q, k, n_traced, epochs, batch_queries, lr, batch_order=None):
    """Train on traces of the exact search; returns (per-step losses, number of pairs)."""
    import numpy as np
    _desc(q, "q")
    nb = (q.shape[0] + batch_queries - 1) // batch_queries
    losses = np.zeros(epochs * nb, dtype=np.float32)
    order = None if batch_order is None else np.ascontiguousarray(batch_order, dtype=np.uint32)
    n = ctypes.c_uint64()
    _check(_lib.qd_model_train(model.handle, tree.handle, _ptr(q), q.shape[0], k, n_traced, epochs, batch_queries,
                               lr, None if order is None else ctypes.c_void_p(order.ctypes.data),
                               ctypes.c_void_p(losses.ctypes.data), ctypes.byref(n), _stream()), "qd_model_train")
    return losses, n.value


# ---------------------------------------------------------------------------
# Batched retrieval plans (hipGraph) and the autotuner
# ---------------------------------------------------------------------------
class _Tuning(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("order", ctypes.c_int), ("waves_per_cu", ctypes.c_uint32),
                ("query_tile", ctypes.c_uint32), ("ms", ctypes.c_float), ("round1_blocks", ctypes.c_uint32),
                ("round2_blocks", ctypes.c_uint32), ("round_growth", ctypes.c_uint32),
                ("round1_start", ctypes.c_uint32)]

    def as_dict(self):
        return {"path": "tree" if self.path else "sequential", "order": self.order,
                "waves_per_cu": self.waves_per_cu, "query_tile": self.query_tile, "ms": self.ms,
                "schedule": (self.round1_blocks, self.round2_blocks, self.round_growth), "start": self.round1_start}


_sig("qd_plan_create", [_P, _P, _U64, _P, _U32, _U64, _U32, _U32, _U32, ctypes.POINTER(_SearchParams), _U32,
                        ctypes.POINTER(ctypes.c_void_p)])
_sig("qd_plan_run", [_P, _P, _U64, _P, _U32, _P, _P, _P, _P])
_sig("qd_plan_free", [_P])
_sig("qd_autotune", [_P, _P, _U64, _P, _U32, _U32, _U32, _U32, ctypes.POINTER(_Tuning), ctypes.POINTER(_Tuning),
                     _U32, ctypes.POINTER(ctypes.c_uint32), _P])


class Plan:
    """A retrieval plan: fixed capacities, buffers allocated once, one batch
    recorded in a hipGraph and replayed per run."""

    def __init__(self, obj_of, n_obj, max_qdesc, max_qobj, k, threshold=10, tree=None, db=None,
                 order=ORDER_BEST_FIRST, waves_per_cu=0, query_tile=0, schedule=(0, 0, 0), start=START_LOWEST_BOUND,
                 model=None, split=0):
        """model (blocked order only): round 1 starts where the model leads.
        split: concurrent subtree searches per query of the per-query orders."""
        if tree is None:
            _desc(db, "db")
        self._keep = (tree, db, obj_of, model)  # the plan points into these
        prm = _SearchParams(order, None, 0, waves_per_cu, None, 0, *schedule)
        prm.round1_start = start
        prm.query_split = split
        if model is not None:
            prm.model = model.handle.value
        h = ctypes.c_void_p()
        _check(_lib.qd_plan_create(tree.handle if tree is not None else None, _ptr(db),
                                   0 if db is None else db.shape[0], _ptr(obj_of), n_obj, max_qdesc, max_qobj, k,
                                   threshold, ctypes.byref(prm), query_tile, ctypes.byref(h)), "qd_plan_create")
        self._h = h
        self.n_obj = n_obj

    def run(self, qdesc, qoff):
        _desc(qdesc, "qdesc")
        nqo = qoff.shape[0] - 1
        dev = qdesc.device
        votes = torch.empty((nqo, self.n_obj), dtype=torch.int32, device=dev)
        winner = torch.empty(nqo, dtype=torch.int32, device=dev)
        used = torch.empty(nqo, dtype=torch.int32, device=dev)
        _check(_lib.qd_plan_run(self._h, _ptr(qdesc), qdesc.shape[0], _ptr(qoff), nqo, _ptr(votes), _ptr(winner),
                                _ptr(used), _stream()), "qd_plan_run")
        return votes, winner, used

    def free(self):
        if self._h is not None and self._h.value:
            _lib.qd_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def autotune(q, k, tree=None, db=None, reps=3, with_all=True, orders=None):
    """(best configuration, all candidates) for a k-NN batch; see qd_autotune.
    orders: the tree frontier orders to time (None = all)."""
    _desc(q, "q")
    best = _Tuning()
    all_ = (_Tuning * 32)()
    n_all = ctypes.c_uint32()
    mask = 0 if orders is None else sum(1 << o for o in orders)
    _check(_lib.qd_autotune(tree.handle if tree is not None else None, _ptr(db), 0 if db is None else db.shape[0],
                            _ptr(q), q.shape[0], k, reps, mask, ctypes.byref(best), all_ if with_all else None, 32,
                            ctypes.byref(n_all), _stream()), "qd_autotune")
    return best.as_dict(), [all_[i].as_dict() for i in range(n_all.value)]
