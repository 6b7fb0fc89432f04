"""Pins for the oracle's sequential k-NN search (Section 6.2's reference).

Checked against special cases that reduce to other definitions (plain Hamming
k-NN via scipy at |q| = 2048; popcount order at |q| = 0 and 4096), planted
neighbours, invariance under permutation of the database, result order and
padding.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import synth

NB = 4096


def _unpack(d):
    return np.unpackbits(np.ascontiguousarray(d).view(np.uint8), axis=1, bitorder="little").astype(bool)


def _pack(bits):
    return np.packbits(bits, axis=1, bitorder="little").view(np.uint64)


def test_half_full_query_is_plain_hamming_knn():
    # With |q| = 2048 both weights are 2048, so K = 2048 * (A + B): the order is
    # the plain Hamming order, which scipy computes on unpacked bits.
    rng = np.random.default_rng(0)
    n, nq, k = 700, 6, 25
    tb = rng.random((n, NB)) < rng.uniform(0.05, 0.95, size=(n, 1))
    qb = np.zeros((nq, NB), bool)
    for j in range(nq):
        qb[j, rng.choice(NB, 2048, replace=False)] = True
    db, q = _pack(tb), _pack(qb)
    r = oracle.knn_brute(db, q, k)
    ham = np.rint(cdist(qb, tb, "hamming") * NB).astype(np.int64)
    for j in range(nq):
        order = np.lexsort((np.arange(n), ham[j]))[:k]
        assert (r.idx[j] == order).all()
        assert (r.missed[j] + r.extra[j] == ham[j, order]).all()


def test_empty_and_full_query_order_by_popcount():
    rng = np.random.default_rng(1)
    n = 300
    tb = rng.random((n, NB)) < rng.uniform(0.0, 1.0, size=(n, 1))
    db = _pack(tb)
    pop = tb.sum(1)
    q = _pack(np.stack([np.zeros(NB, bool), np.ones(NB, bool)]))
    r = oracle.knn_brute(db, q, 12)
    # |q| = 0: only type B errors, K = |t|: sparsest targets first
    assert (r.idx[0] == np.lexsort((np.arange(n), pop))[:12]).all()
    # |q| = 4096: only type A errors, K = 4096 - |t|: densest targets first
    assert (r.idx[1] == np.lexsort((np.arange(n), -pop))[:12]).all()


def test_planted_neighbour_and_sorted_keys(small_db):
    rng = np.random.default_rng(2)
    rows = rng.choice(small_db.shape[0], 10, replace=False)
    r = oracle.knn_brute(small_db, small_db[rows], 10)
    assert (r.idx[:, 0] == rows).all()
    assert (r.missed[:, 0] == 0).all() and (r.extra[:, 0] == 0).all() and (r.dist[:, 0] == 0).all()
    P = _unpack(small_db[rows]).sum(1)
    wa, wb = np.maximum(P, 1), np.maximum(NB - P, 1)
    K = r.missed.astype(np.int64) * wb[:, None] + r.extra.astype(np.int64) * wa[:, None]
    for j in range(10):
        pairs = list(zip(K[j], r.idx[j]))
        assert pairs == sorted(pairs) and len(set(pairs)) == 10


def test_permutation_invariance(small_db, small_queries):
    q, _ = small_queries
    db = small_db[:3000]
    perm = synth.permutation(db.shape[0], 77)
    a = oracle.knn_brute(db, q[:10], 15)
    b = oracle.knn_brute(db[perm], q[:10], 15)
    P = _unpack(q[:10]).sum(1)
    wa, wb = np.maximum(P, 1), np.maximum(NB - P, 1)
    ka = a.missed * wb[:, None] + a.extra * wa[:, None]
    kb = b.missed * wb[:, None] + b.extra * wa[:, None]
    assert (ka == kb).all()
    for j in range(10):
        for s in range(15):
            if (ka[j] == ka[j, s]).sum() == 1:  # unique key: the same row must come back
                assert perm[b.idx[j, s]] == a.idx[j, s]


def test_padding_when_fewer_rows_than_k(small_db):
    r = oracle.knn_brute(small_db[:3], small_db[:2], 5)
    assert (r.idx[:, 3:] == 0xFFFFFFFF).all() and (r.missed[:, 3:] == -1).all()
    assert np.isinf(r.dist[:, 3:]).all() and (r.idx[:, :3] != 0xFFFFFFFF).all()


def test_recall_on_synthetic_queries(small_db, small_queries):
    # sanity of the workload: the source row of a partial query is its nearest neighbour
    q, src = small_queries
    r = oracle.knn_brute(small_db, q, 1)
    assert (r.idx[:, 0] == src).mean() >= 0.95
