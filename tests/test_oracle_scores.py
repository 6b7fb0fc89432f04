"""Pins for the oracle's object-level distance score (Section 6.4): the sum,
over a query object's descriptors, of each one's distance (Eq. 1) to its
nearest descriptor of a database object."""
from fractions import Fraction

import numpy as np

import oracle
import synth

H = 2048  # a half-full descriptor: wA = wB = 2048 and Eq. 1 is Hamming / 2048


def test_hand_worked_scores():
    q1 = list(range(0, H))                  # the first 2048 bits
    q2 = list(range(H, 4096))               # the other 2048
    q3 = list(range(0, 1024))               # |q| = 1024: wA = 1024, wB = 3072
    rows = [
        q1[4:],                             # object 0: Hamming 4 to q1, 4092 to q2
        q2[12:],                            # object 0: Hamming 12 to q2, 4084 to q1
        q1 + list(range(H, H + 52)),        # object 1: Hamming 52 to q1, 4044 to q2
        q1,                                 # object id 3 >= n_obj: belongs to no object
        list(range(4, 1024)) + list(range(1024, 1032)),  # object 1: A = 4, B = 8 for q3
    ]
    db = synth.from_bits(len(rows), rows)
    obj = np.array([0, 0, 1, 3, 1], np.uint16)
    q = synth.from_bits(3, [q1, q2, q3])
    qoff = np.array([0, 2, 2, 3], np.uint64)   # {q1, q2}, {}, {q3}
    s = oracle.object_scores(db, obj, 3, q, qoff)
    # {q1, q2}: object 0 gives 4/2048 + 12/2048.  Object 1: q1 is 52 from row 2
    # and 1020 (bits 0..3 and 1032..2047) from row 4; q2 is 4044 from row 2 and
    # 3076 (all of q2 and the 1028 bits of row 4) from row 4: (52 + 3076) / 2048
    assert s[0].tolist() == [16 / H, 3128 / H, np.inf]
    # the empty query object scores 0 everywhere, an object without rows included
    assert s[1].tolist() == [0.0, 0.0, 0.0]
    # {q3}: object 1's last row, A/|q| + B/(4096-|q|) = 4/1024 + 8/3072 = 5/768
    assert s[2][1] == float(Fraction(5, 768))
    # row 0 = bits 4..2047: A = 4 (bits 0..3), B = 1024 (bits 1024..2047)
    # row 1 = bits 2060..4095: A = 1024, B = 2036; row 0 is nearer
    assert s[2][0] == float(Fraction(4, 1024) + Fraction(1024, 3072))
    assert s[2][2] == np.inf


def _exact(q, t):
    A, B, P = oracle.wh_literal(q, t)
    wa, wb = max(P, 1), max(4096 - P, 1)
    return float(Fraction(A * wb + B * wa, wa * wb))


def _setup(n_obj=12, per=150, nqo=10, seed=51):
    db = synth.gen_db(n_obj * per, seed)
    perm = synth.permutation(n_obj * per, seed + 1)
    obj = (perm % n_obj).astype(np.uint16)           # objects interleaved in the rows
    off, src, qobj = synth.gen_query_objects(n_obj, per, nqo, seed + 2, 3, 9)
    # gen_query_objects numbers object o's rows o*per .. o*per+per-1; map them
    # to the interleaved layout: the j-th row of object o
    rows_of = [np.flatnonzero(obj == o) for o in range(n_obj)]
    src = np.array([rows_of[r // per][r % per] for r in src], np.uint32)
    q, _ = synth.gen_queries(db, len(src), seed + 3, 0.2, 0.5, src=src)
    return db, obj, n_obj, q, off, qobj


def test_single_descriptor_reduces_to_nearest_neighbour():
    # a one-descriptor query object scores, against object o, the distance of
    # its first neighbour in object o's rows (the k-NN routine on the subset)
    db, obj, n_obj, q, _, _ = _setup()
    q = q[:6]
    s = oracle.object_scores(db, obj, n_obj, q, np.arange(len(q) + 1, dtype=np.uint64))
    for o in range(n_obj):
        sub = db[obj == o]
        nn = oracle.knn_brute(sub, q, 1)
        for g in range(len(q)):
            assert s[g, o] == _exact(q[g], sub[nn.idx[g, 0]])


def test_sum_in_descriptor_order():
    db, obj, n_obj, q, off, _ = _setup()
    single = oracle.object_scores(db, obj, n_obj, q, np.arange(len(q) + 1, dtype=np.uint64))
    s = oracle.object_scores(db, obj, n_obj, q, off)
    for g in range(len(off) - 1):
        acc = np.zeros(n_obj)
        for d in range(int(off[g]), int(off[g + 1])):
            acc = acc + single[d]
        assert np.array_equal(s[g], acc)


def test_exact_copies_score_zero_and_source_object_ranks_first():
    db, obj, n_obj, q, off, qobj = _setup()
    # unmodified copies of object 3's rows score 0 against it, > 0 elsewhere
    copies = db[obj == 3][:5]
    s0 = oracle.object_scores(db, obj, n_obj, copies, np.array([0, 5], np.uint64))[0]
    assert s0[3] == 0.0 and (np.delete(s0, 3) > 0).all()
    # partial noisy copies: the source object has the lowest total distance
    s = oracle.object_scores(db, obj, n_obj, q, off)
    assert (s >= 0).all()
    assert (s.argmin(1) == qobj).all()


def test_row_permutation_invariance():
    db, obj, n_obj, q, off, _ = _setup()
    s = oracle.object_scores(db, obj, n_obj, q, off)
    p = synth.permutation(len(db), 77)
    assert np.array_equal(oracle.object_scores(db[p], obj[p], n_obj, q, off), s)


def test_score_rows_hand_worked():
    s = np.array([[3.0, 1.0, np.inf, 2.0],
                  [2.0, 1.0, 1.0, 4.0],        # tie: the lower id wins
                  [np.inf, np.inf, np.inf, np.inf],
                  [5.0, 5.0, np.inf, 5.0]])
    best, norm = oracle.score_rows(s)
    assert best.tolist() == [1, 1, -1, 0]
    assert norm.tolist() == [[1.0, 0.0, 1.0, 0.5],
                             [1 / 3, 0.0, 0.0, 1.0],
                             [1.0, 1.0, 1.0, 1.0],
                             [0.0, 0.0, 1.0, 0.0]]
    best2, same = oracle.score_rows(s, normalize=False)
    assert best2.tolist() == best.tolist() and np.array_equal(same, s)


def test_score_rows_properties():
    db, obj, n_obj, q, off, qobj = _setup()
    s = oracle.object_scores(db, obj, n_obj, q, off)
    best, norm = oracle.score_rows(s)
    assert np.array_equal(best, s.argmin(1))            # first minimum = lowest id
    assert (norm.min(1) == 0).all() and (norm.max(1) == 1).all()
    for g in range(len(s)):                             # the order of the objects is kept
        assert np.array_equal(np.argsort(norm[g], kind="stable"), np.argsort(s[g], kind="stable"))
    # a scale by a power of two changes no bit of the normalised rows
    assert np.array_equal(oracle.score_rows(4 * s)[1], norm)
