"""Pins for the oracle's vote aggregation (Section 3's pipeline)."""
import numpy as np

import oracle
import synth


def test_hand_worked_votes():
    # 6 database rows owned by objects [0, 0, 1, 1, 2, 2]; threshold 2.
    obj = np.array([0, 0, 1, 1, 2, 2], np.uint16)
    # query object 0: neighbours (k = 2) per descriptor in processing order
    #   d0 -> rows 2, 4   votes: o1=1, o2=1
    #   d1 -> rows 0, 3   votes: o0=1, o1=2  <- o1 reaches 2 first (descriptor 2 of 3)
    #   d2 -> rows 5, 4   votes: o2=3
    # query object 1: one descriptor, rows 1 and padding -> o0 = 1, no winner
    nn = np.array([[2, 4], [0, 3], [5, 4], [1, 0xFFFFFFFF]], np.uint32)
    qoff = np.array([0, 3, 4], np.uint64)
    v, w, u = oracle.votes(nn, obj, 3, qoff, threshold=2)
    assert v.tolist() == [[1, 2, 3], [1, 0, 0]]
    assert w.tolist() == [1, -1]
    assert u.tolist() == [2, 1]


def test_vote_totals_and_planted_object():
    n_obj, per = 20, 200
    db = synth.gen_db(n_obj * per, 41)
    obj = (np.arange(n_obj * per) // per).astype(np.uint16)
    off, rows, qobj = synth.gen_query_objects(n_obj, per, 6, 42, 15, 40)
    # zero partiality, zero flips: each query descriptor is its own source row
    q, _ = synth.gen_queries(db, len(rows), 43, 0.0, 0.0, nflip=0, src=rows)
    nn = oracle.knn_brute(db, q, 3)
    v, w, u = oracle.votes(nn.idx, obj, n_obj, off, threshold=10)
    assert (v.sum(1) == 3 * np.diff(off)).all()
    assert (w == qobj).all()
    # with every first neighbour in the right object, the winner needs at most 10 descriptors
    assert (u <= 10).all()


def test_rows_of_no_object_cast_no_vote():
    # rows 1 and 3 carry ids 7 and 3, both >= n_obj = 3: they belong to no object
    obj = np.array([0, 7, 1, 3, 2, 2], np.uint16)
    #   d0 -> rows 1, 0   votes: o0=1 (row 1 casts none)
    #   d1 -> rows 3, 0   votes: o0=2  <- o0 reaches 2 at descriptor 2
    #   d2 -> rows 1, 3   no votes
    nn = np.array([[1, 0], [3, 0], [1, 3]], np.uint32)
    v, w, u = oracle.votes(nn, obj, 3, np.array([0, 3], np.uint64), threshold=2)
    assert v.tolist() == [[2, 0, 0]]
    assert w.tolist() == [0] and u.tolist() == [2]
    # no object reaches the threshold when only rows of no object are found
    v, w, u = oracle.votes(nn[2:], obj, 3, np.array([0, 1], np.uint64), threshold=1)
    assert v.tolist() == [[0, 0, 0]] and w.tolist() == [-1] and u.tolist() == [1]
