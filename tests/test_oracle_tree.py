"""Pins for the oracle's Dissimilarity Tree build (Listing 1) and query (Listing 2).

Hand-worked splits fix the reading of the move loop; an independent
characterisation of every split (the dissimilar side is exactly the rows whose
least popular set bit ranks at or below a cut, with the cut at the first
point where half the node has moved) is checked at every node of a 10k tree;
the tree search must return exactly the brute-force result, and the node
bound must never exceed the key of any row under the node.
"""
import numpy as np
import pytest

import oracle
import synth

NB = 4096


def _unpack(d):
    return np.unpackbits(np.ascontiguousarray(d).view(np.uint8), axis=1, bitorder="little").astype(bool)


def test_hand_split_stops_at_half():
    # 40 rows: bit 100 in all, bit 200 in rows 0-4, bit 300 in rows 5-24, bit 400 in rows 25-39.
    # Ascending popularity: 200 (5), 400 (15), 300 (20), 100 (40).  Moving 200 gives 5 rows,
    # then 400 gives 20 = half of 40: stop.  Similar = rows 5-24, dissimilar = 0-4 and 25-39.
    bits = []
    for i in range(40):
        b = [100]
        b.append(200 if i < 5 else (300 if i < 25 else 400))
        bits.append(b)
    db = synth.from_bits(40, bits)
    side = oracle.split_node(db, np.arange(40))
    assert (np.flatnonzero(side) == np.r_[0:5, 25:40]).all()
    t = oracle.tree_build(db, max_leaf=32)
    assert t.n_nodes == 3
    assert (t.child[0] == [1, 2]).all() and (t.child[1:] == -1).all()
    assert list(t.begin) == [0, 0, 20] and list(t.count) == [40, 20, 20]
    assert (t.perm == np.r_[5:25, 0:5, 25:40]).all()


def test_hand_split_never_empties_similar():
    # 34 rows all with bit 10, rows 0-1 also with bit 20.  Bit 20 moves 2 rows; bit 10
    # would move all 32 remaining rows, which would empty the similar set: not applied.
    bits = [[10, 20] if i < 2 else [10] for i in range(34)]
    db = synth.from_bits(34, bits)
    side = oracle.split_node(db, np.arange(34))
    assert (np.flatnonzero(side) == [0, 1]).all()
    t = oracle.tree_build(db)
    assert list(t.count) == [34, 32, 2]


def test_degenerate_nodes_become_leaves():
    same = synth.from_bits(40, [[1, 2, 3]] * 40)
    t = oracle.tree_build(same)
    assert t.n_nodes == 1 and t.count[0] == 40
    zero = np.zeros((40, 64), np.uint64)
    assert oracle.tree_build(zero).n_nodes == 1
    # zero rows never move; when every set bit is used and under half moved, the
    # nonzero rows form the dissimilar side
    mixed = synth.from_bits(40, [[] for _ in range(30)] + [[5]] * 10)
    t = oracle.tree_build(mixed)
    assert list(t.count) == [40, 30, 10] and (t.perm[30:] == np.arange(30, 40)).all()


def _check_split(db_bits, members, sim, dis):
    n = len(members)
    cnt = db_bits[members].sum(0)
    order = np.lexsort((np.arange(NB), cnt))
    rank = np.empty(NB, np.int64)
    rank[order] = np.arange(NB)
    big = NB + 1
    fr = np.where(db_bits[members], rank[None, :], big).min(1)  # rank of least popular set bit
    in_d = np.zeros(n, bool)
    in_d[np.searchsorted(members, dis)] = True
    jcut = fr[in_d].max()
    assert (in_d == (fr <= jcut)).all()          # dissimilar = rows moved by bits up to the cut
    assert 2 * (fr < jcut).sum() < n             # it had not reached half before the cut
    if 2 * in_d.sum() < n:                       # stopped short of half: the next move empties S
        rest = fr[~in_d]
        assert (rest == rest.min()).all()


def test_every_split_of_a_10k_tree(small_db):
    t = oracle.tree_build(small_db, max_leaf=32)
    bits = _unpack(small_db)
    n = small_db.shape[0]
    assert sorted(t.perm.tolist()) == list(range(n))
    leaves = 0
    for i in range(t.n_nodes):
        b, c = t.begin[i], t.count[i]
        mem = np.sort(t.perm[b:b + c])
        assert (np.bitwise_or.reduce(small_db[mem], axis=0) == t.or_img[i]).all()
        assert (np.bitwise_and.reduce(small_db[mem], axis=0) == t.and_img[i]).all()
        s, d = t.child[i]
        if s < 0:
            leaves += 1
            assert (t.perm[b:b + c] == mem).all()  # stable partitions keep ascending row order
            assert c <= 32 or (small_db[mem] == small_db[mem[0]]).all()
            continue
        assert t.begin[s] == b and t.begin[d] == b + t.count[s] and t.count[s] + t.count[d] == c
        assert s > i and d == s + 1
        assert (t.or_img[s] | t.or_img[d] == t.or_img[i]).all()
        _check_split(bits, mem, np.sort(t.perm[b:b + t.count[s]]), np.sort(t.perm[t.begin[d]:b + c]))
    assert leaves == (t.child[:, 0] < 0).sum() and leaves * 2 - 1 == t.n_nodes


@pytest.mark.parametrize("k", [1, 10, 50])
def test_tree_search_equals_bruteforce(small_db, small_queries, k):
    q, _ = small_queries
    t = oracle.tree_build(small_db)
    a = oracle.knn_brute(small_db, q, k)
    b = oracle.tree_knn(small_db, t, q, k)
    c = oracle.tree_knn(small_db, t, q, k, use_and=True)
    d = oracle.tree_knn(small_db, t, q, k, use_pop=True)
    e = oracle.tree_knn(small_db, t, q, k, use_and=True, use_pop=True)
    for r in (b, c, d, e):
        assert (a.idx == r.idx).all() and (a.missed == r.missed).all() and (a.extra == r.extra).all()
        assert (a.dist == r.dist).all()
    assert (b.stats[:, 2] < small_db.shape[0]).mean() > 0.5  # the tree prunes on this data
    assert (c.stats[:, 0] <= b.stats[:, 0]).all()              # the product image only tightens
    assert d.stats[:, 0].sum() < b.stats[:, 0].sum()           # so does the popcount range
    assert e.stats[:, 0].sum() <= d.stats[:, 0].sum()


def test_bound_never_exceeds_any_key():
    db = synth.gen_db(600, 31)
    q, _ = synth.gen_queries(db, 6, 32, 0.1, 0.6)
    t = oracle.tree_build(db, max_leaf=8)
    r = oracle.knn_brute(db, q, 600)
    P = _unpack(q).sum(1)
    wa, wb = np.maximum(P, 1), np.maximum(NB - P, 1)
    pmin, pmax = oracle.node_pop_range(db, t)
    tighter = 0
    for j in range(len(q)):
        key = np.empty(600, np.int64)
        key[r.idx[j]] = r.missed[j].astype(np.int64) * wb[j] + r.extra[j].astype(np.int64) * wa[j]
        for i in range(t.n_nodes):
            rows = t.perm[t.begin[i]:t.begin[i] + t.count[i]]
            lb = oracle.node_bound(q[j], t.or_img[i])
            lb2 = oracle.node_bound(q[j], t.or_img[i], t.and_img[i])
            pr = (pmin[i], pmax[i])
            lb3 = oracle.node_bound(q[j], t.or_img[i], pop_range=pr)
            lb4 = oracle.node_bound(q[j], t.or_img[i], t.and_img[i], pop_range=pr)
            assert lb <= lb2 <= lb4 <= key[rows].min()
            assert lb <= lb3 <= lb4
            tighter += lb3 > lb


    assert tighter > 0  # the popcount terms take part


def test_popcount_range_bound_hand_worked():
    # |q| = 100 (bits 0..99): wA = 100, wB = 3996
    q = synth.from_bits(1, [range(100)])[0]
    # rows of 10 and 12 bits, both disjoint from q: ov = 0, so A >= 100 and
    # B >= pmin = 10; the 10-bit row reaches the bound exactly
    rows = synth.from_bits(2, [range(200, 210), range(300, 312)])
    img = rows[0] | rows[1]
    assert oracle.node_bound(q, img) == 100 * 3996
    assert oracle.node_bound(q, img, pop_range=(10, 12)) == 100 * 3996 + 10 * 100
    # eight rows of 5 bits inside q's bits 0..39: the image covers 40 query
    # bits (ov = 40) but no row more than 5, so A >= 95; every row reaches it
    rows = synth.from_bits(8, [range(5 * i, 5 * i + 5) for i in range(8)])
    img = np.bitwise_or.reduce(rows, axis=0)
    assert oracle.node_bound(q, img) == 60 * 3996
    assert oracle.node_bound(q, img, pop_range=(5, 5)) == 95 * 3996
    # the product image's B term and the popcount term, the larger counts:
    # rows of 40 bits outside q sharing 10 of them; B >= max(10, 40 - 0)
    rows = synth.from_bits(2, [list(range(200, 210)) + list(range(300, 330)),
                               list(range(200, 210)) + list(range(400, 430))])
    img, and_img = rows[0] | rows[1], rows[0] & rows[1]
    assert oracle.node_bound(q, img, and_img) == 100 * 3996 + 10 * 100
    assert oracle.node_bound(q, img, and_img, pop_range=(40, 40)) == 100 * 3996 + 40 * 100


def test_any_frontier_order_gives_the_same_result(small_db, small_queries):
    q, _ = small_queries
    q = q[:20]
    t = oracle.tree_build(small_db)
    plain = oracle.tree_knn(small_db, t, q, 10)
    rng = np.random.default_rng(4)
    for score in (rng.integers(0, 1 << 40, size=(len(q), t.n_nodes)),
                  np.zeros((len(q), t.n_nodes), np.int64),
                  -np.tile(np.arange(t.n_nodes), (len(q), 1))):
        r = oracle.tree_knn(small_db, t, q, 10, score=score)
        assert (r.idx == plain.idx).all() and (r.dist == plain.dist).all()
