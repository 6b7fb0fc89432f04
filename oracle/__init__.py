"""CPU oracle for Weighted Hamming k-NN over 64x64-bit QUICCI descriptors.

TEST INFRASTRUCTURE ONLY.  The plain, slow reference the GPU library is
checked against; only the tests, the smoke check and the benchmark's CPU
baseline may import it.  It shares no code with the GPU library and imports
nothing from it.

Functions take numpy arrays: descriptors are ``uint64`` of shape ``(n, 64)``
(word r = image row r, bit c = column c).
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

NBITS = 4096
PAD_IDX = 0xFFFFFFFF


def build():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO,
                           os.path.join(_HERE, "oracle.c")])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        lib.or_wh_literal.argtypes = [P, P, P, P, P]
        lib.or_wh_eq1.argtypes = [I64, I64, I64]
        lib.or_wh_eq1.restype = ctypes.c_double
        lib.or_wh_key.argtypes = [I64, I64, I64]
        lib.or_wh_key.restype = I64
        lib.or_wh_dist.argtypes = [I64, I64, I64]
        lib.or_wh_dist.restype = ctypes.c_float
        lib.or_knn_brute.argtypes = [P, I64, P, I64, I, P, P, P, P]
        lib.or_split_node.argtypes = [P, P, I64, P]
        lib.or_split_node.restype = I64
        lib.or_tree_build.argtypes = [P, I64, I, I64, P, P, P, P, P, P]
        lib.or_tree_build.restype = I64
        lib.or_node_bound.argtypes = [P, P, P]
        lib.or_node_bound.restype = I64
        lib.or_node_bound_pop.argtypes = [P, P, P, I64, I64]
        lib.or_node_bound_pop.restype = I64
        lib.or_tree_knn.argtypes = [P, P, P, P, P, P, P, P, P, I64, P, I64, I, P, P, P, P, P, P]
        lib.or_votes.argtypes = [P, I, P, I64, I64, P, I64, I64, P, P, P]
        lib.or_object_scores.argtypes = [P, I64, P, I64, P, P, I64, P]
        lib.or_score_rows.argtypes = [P, I64, I64, I, P]
        lib.or_set_threads.argtypes = [I]
        lib.or_max_threads.restype = I
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _desc(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if a.ndim == 1:
        a = a.reshape(1, 64)
    assert a.shape[1] == 64
    return a


def wh_literal(q, t):
    """(A, B, |q|) of Eq. 1 by the row/column loop."""
    lib = _load()
    q = _desc(q)
    t = _desc(t)
    out = np.zeros(3, dtype=np.int64)
    lib.or_wh_literal(_p(q), _p(t), _p(out[0:]), _p(out[1:]), _p(out[2:]))
    return int(out[0]), int(out[1]), int(out[2])


def wh_eq1(A, B, P):
    return _load().or_wh_eq1(A, B, P)


def wh_key(A, B, P):
    return _load().or_wh_key(A, B, P)


def wh_dist(A, B, P):
    return _load().or_wh_dist(A, B, P)


@dataclass
class Knn:
    idx: np.ndarray
    missed: np.ndarray
    extra: np.ndarray
    dist: np.ndarray
    stats: np.ndarray = None  # (nq, 3): nodes visited, bounds, distances (tree search only)


def knn_brute(db, q, k):
    lib = _load()
    db = _desc(db)
    q = _desc(q)
    nq = q.shape[0]
    out = Knn(np.empty((nq, k), np.uint32), np.empty((nq, k), np.int32), np.empty((nq, k), np.int32),
              np.empty((nq, k), np.float32))
    rc = lib.or_knn_brute(_p(db), db.shape[0], _p(q), nq, k, _p(out.idx), _p(out.missed), _p(out.extra),
                          _p(out.dist))
    assert rc == 0
    return out


@dataclass
class Tree:
    n_nodes: int
    child: np.ndarray    # int32 (n_nodes, 2): similar, dissimilar; -1 for a leaf
    begin: np.ndarray    # int64 (n_nodes,)
    count: np.ndarray    # int64 (n_nodes,)
    or_img: np.ndarray   # uint64 (n_nodes, 64) sum image
    and_img: np.ndarray  # uint64 (n_nodes, 64) product image
    perm: np.ndarray     # uint32 (n,) database rows in leaf order


def split_node(db, members):
    """Listing 1's split of one node: boolean array, True = dissimilar."""
    lib = _load()
    db = _desc(db)
    mem = np.ascontiguousarray(members, dtype=np.uint32)
    side = np.zeros(len(mem), dtype=np.uint8)
    lib.or_split_node(_p(db), _p(mem), len(mem), _p(side))
    return side.astype(bool)


def tree_build(db, max_leaf=32):
    lib = _load()
    db = _desc(db)
    n = db.shape[0]
    cap = 2 * n + 1
    child = np.empty((cap, 2), np.int32)
    begin = np.empty(cap, np.int64)
    count = np.empty(cap, np.int64)
    or_img = np.empty((cap, 64), np.uint64)
    and_img = np.empty((cap, 64), np.uint64)
    perm = np.empty(n, np.uint32)
    nn = lib.or_tree_build(_p(db), n, max_leaf, cap, _p(child), _p(begin), _p(count), _p(or_img), _p(and_img),
                           _p(perm))
    assert nn > 0
    return Tree(nn, child[:nn].copy(), begin[:nn].copy(), count[:nn].copy(), or_img[:nn].copy(),
                and_img[:nn].copy(), perm)


def node_bound(q, or_img, and_img=None, pop_range=None):
    """Lower bound on the key of every row under a node; pop_range = (pmin,
    pmax) of the node's rows adds the popcount-range terms."""
    lib = _load()
    a = None if and_img is None else _desc(and_img)
    if pop_range is not None:
        return lib.or_node_bound_pop(_p(_desc(q)), _p(_desc(or_img)), _p(a), int(pop_range[0]), int(pop_range[1]))
    return lib.or_node_bound(_p(_desc(q)), _p(_desc(or_img)), _p(a))


def node_pop_range(db, tree):
    """(pmin, pmax) per node: the smallest and largest popcount of its rows."""
    db = _desc(db)
    pop = np.unpackbits(db.view(np.uint8), axis=1).sum(1).astype(np.int64)[tree.perm]
    pmin = np.array([pop[b:b + c].min() for b, c in zip(tree.begin, tree.count)], np.int64)
    pmax = np.array([pop[b:b + c].max() for b, c in zip(tree.begin, tree.count)], np.int64)
    return pmin, pmax


def tree_knn(db, tree, q, k, use_and=False, score=None, use_pop=False):
    """Best-first k-NN over ``tree``.  ``score`` (nq, n_nodes) int64 replaces
    the bound as the frontier order (results must not change); ``use_pop``
    tightens the bound with each node's popcount range."""
    lib = _load()
    db = _desc(db)
    q = _desc(q)
    nq = q.shape[0]
    child = np.ascontiguousarray(tree.child, np.int32)
    begin = np.ascontiguousarray(tree.begin, np.int64)
    count = np.ascontiguousarray(tree.count, np.int64)
    or_img = np.ascontiguousarray(tree.or_img, np.uint64)
    and_img = np.ascontiguousarray(tree.and_img, np.uint64) if use_and else None
    pmin, pmax = node_pop_range(db, tree) if use_pop else (None, None)
    perm = np.ascontiguousarray(tree.perm, np.uint32)
    sc = None if score is None else np.ascontiguousarray(score, np.int64)
    out = Knn(np.empty((nq, k), np.uint32), np.empty((nq, k), np.int32), np.empty((nq, k), np.int32),
              np.empty((nq, k), np.float32), np.empty((nq, 3), np.int64))
    rc = lib.or_tree_knn(_p(db), _p(child), _p(begin), _p(count), _p(or_img), _p(and_img), _p(pmin), _p(pmax),
                         _p(perm), tree.n_nodes, _p(q), nq, k, _p(sc), _p(out.idx), _p(out.missed), _p(out.extra),
                         _p(out.dist), _p(out.stats))
    assert rc == 0
    return out


def set_threads(n):
    """Threads the oracle's parallel loops use from now on (timing only)."""
    _load().or_set_threads(int(n))


def max_threads():
    return _load().or_max_threads()


def votes(nn_idx, obj_of, n_obj, qoff, threshold=10):
    """Vote histogram, winner and descriptors used per query object."""
    lib = _load()
    nn_idx = np.ascontiguousarray(nn_idx, np.uint32)
    k = nn_idx.shape[1]
    obj_of = np.ascontiguousarray(obj_of, np.uint16)
    qoff = np.ascontiguousarray(qoff, np.uint64)
    nqo = len(qoff) - 1
    v = np.empty((nqo, n_obj), np.uint32)
    w = np.empty(nqo, np.int32)
    u = np.empty(nqo, np.uint32)
    lib.or_votes(_p(nn_idx), k, _p(obj_of), len(obj_of), n_obj, _p(qoff), nqo, threshold, _p(v), _p(w), _p(u))
    return v, w, u


def object_scores(db, obj_of, n_obj, q, qoff):
    """Summed nearest-neighbour distance of every query object to every
    database object (nqo x n_obj float64; +inf for objects without rows)."""
    lib = _load()
    db = _desc(db)
    q = _desc(q) if len(q) else np.zeros((0, 64), np.uint64)
    obj_of = np.ascontiguousarray(obj_of, np.uint16)
    qoff = np.ascontiguousarray(qoff, np.uint64)
    nqo = len(qoff) - 1
    out = np.empty((nqo, n_obj), np.float64)
    lib.or_object_scores(_p(db), len(db), _p(obj_of), n_obj, _p(q), _p(qoff), nqo, _p(out))
    return out


def score_rows(scores, normalize=True):
    """Best object per row (lowest score, ties to the lower id, -1 if none is
    finite) and, with normalize, the rows rescaled to [0, 1] (a copy)."""
    lib = _load()
    s = np.array(scores, dtype=np.float64, order="C", copy=True)
    nqo, n_obj = s.shape
    best = np.empty(nqo, np.int32)
    lib.or_score_rows(_p(s), nqo, n_obj, 1 if normalize else 0, _p(best))
    return best, s

