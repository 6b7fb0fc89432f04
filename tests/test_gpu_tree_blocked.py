"""Batched (blocked) tree search on the matrix cores against the CPU oracle.

The blocked order must return the sequential-search result bit for bit: at
sizes that span several rounds, several query tiles per block and a ragged
last block; on degenerate inputs; when candidate buffers overflow (the
per-query fallback); across query batches; and at 1M rows, where every query
is compared with the per-query best-first search and sampled ones with the
oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qd():
    import paper_2107_03368_amd as qd
    return qd


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda:0")


def _np(res):
    idx, missed, extra, dist = (x.cpu().numpy() for x in res[:4])
    return idx.view(np.uint32), missed, extra, dist


def _same(res, ref, rows=None):
    idx, missed, extra, dist = _np(res)
    if rows is not None:
        idx, missed, extra, dist = idx[rows], missed[rows], extra[rows], dist[rows]
    assert np.array_equal(idx, ref.idx)
    assert np.array_equal(missed, ref.missed)
    assert np.array_equal(extra, ref.extra)
    assert np.array_equal(dist, ref.dist)

def _sample(fixed, nq, seed, extra=59):
    """Query rows the oracle checks: the given ones and `extra` more at random."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.array(fixed), rng.choice(nq, extra, replace=False)]))



@pytest.mark.parametrize("k", [1, 10, 50])
def test_blocked_matches_oracle_10k(qd, small_db, small_queries, k):
    q, _ = small_queries
    tree = qd.tree_build(_t(small_db))
    ref = oracle.knn_brute(small_db, q, k)
    _same(qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED), ref)


@pytest.mark.parametrize("k", [1, 10, 64])
def test_blocked_several_rounds_and_tiles(qd, k):
    # 60,123 rows: 235 blocks, the last one ragged; 600 queries: up to three
    # 256-query tiles per block; the round schedule 16, 64, 128, all.
    db = synth.gen_db(60_123, 1101)
    q, _ = synth.gen_queries(db, 600, 2101, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    ref = oracle.knn_brute(db, q, k)
    res = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, query_stats=True, totals=True)
    _same(res, ref)
    st = res[4].cpu().numpy()
    nblk = (db.shape[0] + 255) // 256
    assert (st[:, 0] >= 16).all() and (st[:, 0] <= nblk).all()   # blocks evaluated
    assert (st[:, 1] >= 1).all()                                # rounds
    assert (st[:, 2] == nblk).all()                             # blocks bounded
    # round 1 alone evaluates 16 blocks (one of them may be the ragged last block)
    assert (st[:, 3] <= db.shape[0]).all() and (st[:, 3] >= 15 * 256 + db.shape[0] % 256).all()
    if k == 1:
        assert st[:, 3].mean() < 0.9 * db.shape[0]  # the bounds prune


@pytest.mark.parametrize("schedule", [(4, 0, 2), (16, 0, 4), (16, 2000, 8), (64, 0, 2)])
def test_blocked_schedules(qd, schedule):
    db = synth.gen_db(60_123, 1101)
    q, _ = synth.gen_queries(db, 600, 2101, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    for k in (1, 10):
        _same(qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, schedule=schedule), oracle.knn_brute(db, q, k))


@pytest.mark.parametrize("k,schedule", [(1, (0, 0, 0)), (10, (0, 0, 0)), (10, (4, 0, 2)), (50, (64, 0, 2)),
                                        (64, (1, 100_000, 2))])
def test_blocked_bound_descent_start(qd, k, schedule):
    # round 1 at the consecutive blocks the bound's descent reaches; the last
    # case overflows round 2 and repeats it with round 1's blocks still done
    db = synth.gen_db(60_123, 1101)
    q, _ = synth.gen_queries(db, 600, 2101, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    res = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, schedule=schedule, start=qd.START_BOUND_DESCENT,
                      query_stats=True)
    _same(res, oracle.knn_brute(db, q, k))
    plain = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, schedule=schedule, query_stats=True)
    assert (plain[4].cpu().numpy() != res[4].cpu().numpy()).any()  # another start: other work, same results


def test_blocked_overflow_repeat(qd):
    # one block in round 1 gives a loose 64th key, and round 2 takes every
    # block: more rows than a candidate buffer holds pass the key, so the
    # queries repeat round 2 with the 64th of the candidates they stored
    db = synth.gen_db(60_123, 1101)
    q, _ = synth.gen_queries(db, 200, 2103, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    res = qd.knn_tree(tree, _t(q), 64, order=qd.ORDER_BLOCKED, schedule=(1, 100_000, 2), query_stats=True)
    _same(res, oracle.knn_brute(db, q, 64))
    assert (res[4].cpu().numpy()[:, 1] >= 3).mean() > 0.5  # most queries repeated a round


def test_blocked_edge_cases(qd):
    base = synth.gen_db(500, 71)
    db = np.concatenate([base, base[:100], np.zeros((5, 64), np.uint64)])
    q = np.concatenate([base[:10], np.zeros((1, 64), np.uint64), np.full((1, 64), np.uint64(0xFFFFFFFFFFFFFFFF)),
                        synth.gen_queries(base, 8, 72, 0.2, 0.6)[0]])
    tree = qd.tree_build(_t(db))
    for k in (1, 7, 64):
        _same(qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED), oracle.knn_brute(db, q, k))
    small = synth.gen_db(3, 73)  # fewer rows than k: padded results
    _same(qd.knn_tree(qd.tree_build(_t(small)), _t(q), 5, order=qd.ORDER_BLOCKED), oracle.knn_brute(small, q, 5))
    one = synth.gen_db(1, 74)
    _same(qd.knn_tree(qd.tree_build(_t(one)), _t(q), 1, order=qd.ORDER_BLOCKED), oracle.knn_brute(one, q, 1))


@pytest.mark.parametrize("plain_bound", [False, True])
def test_blocked_degenerate_queries_on_the_matrix_cores(qd, plain_bound):
    # block lists long enough (>= 24 queries, above the short-list cutoff) for the matrix-core tiles, made
    # of degenerate queries only: all zero (|q| = 0: every block's bound is 0,
    # the key is the row's popcount), all one (|q| = 4096), one set bit, and
    # all but one bit; the rows include all-zero, all-one and dense rows
    db = synth.gen_db(60_123, 1104)
    rng = np.random.default_rng(1105)
    at = rng.choice(len(db), 60, replace=False)
    db[at[:20]] = 0
    db[at[20:40]] = np.uint64(0xFFFFFFFFFFFFFFFF)
    db[at[40:]] = rng.integers(0, 2 ** 63, (20, 64), dtype=np.int64).view(np.uint64)
    one_bit = np.zeros((40, 64), np.uint64)
    one_bit[np.arange(40), rng.integers(0, 64, 40)] = np.uint64(1) << rng.integers(0, 64, 40).astype(np.uint64)
    all_but = ~one_bit
    q = np.concatenate([np.zeros((40, 64), np.uint64), np.full((40, 64), np.uint64(0xFFFFFFFFFFFFFFFF)),
                        one_bit, all_but])
    tree = qd.tree_build(_t(db), plain_bound=plain_bound)
    for k in (1, 10, 64):
        ref = oracle.knn_brute(db, q, k)
        qd.profile_enable(True)
        res = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED)
        tiles = qd.profile_counter("tree_block_tiles")
        qd.profile_enable(False)
        _same(res, ref)
        assert tiles > 0
        _same(qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, start=qd.START_BOUND_DESCENT), ref)


def test_blocked_overflow_fallback(qd):
    # 30,000 copies of one descriptor: after round 1 the k-th key equals the
    # copies' key, so round 2 appends every copy of its blocks (more than a
    # candidate buffer holds) and the queries are searched again best-first.
    rng_db = synth.gen_db(4000, 75)
    dup = np.repeat(rng_db[:1], 30_000, axis=0)
    db = np.concatenate([rng_db, dup])
    q = np.concatenate([rng_db[:3], synth.gen_queries(rng_db, 5, 76, 0.2, 0.5)[0]])
    tree = qd.tree_build(_t(db))
    for k in (1, 10):
        _same(qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED), oracle.knn_brute(db, q, k))


def test_blocked_several_batches(qd):
    # more queries than one batch holds (16,384)
    db = synth.gen_db(5_000, 1102)
    q, _ = synth.gen_queries(db, 16_500, 2102, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    res = qd.knn_tree(tree, _t(q), 10, order=qd.ORDER_BLOCKED)
    ref_gpu = qd.knn_bruteforce(_t(db), _t(q), 10)
    for a, b in zip(_np(res), _np(ref_gpu)):
        assert np.array_equal(a, b)
    rows = _sample([0, 1, 16_383, 16_384, 16_499], 16_500, 33)
    _same(res, oracle.knn_brute(db, q[rows], 10), rows)


@pytest.fixture(scope="module")
def tree_1m(qd):
    db = synth.gen_db(1_000_000, 1001)
    return db, qd.tree_build(_t(db))


@pytest.mark.parametrize("k", [1, 10, 50])
def test_blocked_1m(qd, tree_1m, k):
    db, tree = tree_1m
    q, _ = synth.gen_queries(db, 4096, 2001, 0.1, 0.6)
    res = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED)
    best = qd.knn_tree(tree, _t(q), k)
    for a, b in zip(_np(res), _np(best)):
        assert np.array_equal(a, b)
    rows = _sample([0, 7, 2048, 4095], 4096, 34)
    _same(res, oracle.knn_brute(db, q[rows], k), rows)


@pytest.mark.parametrize("k", [1, 10])
def test_blocked_popcount_range_and_plain_bound(qd, k):
    # blocks bounded with their rows' popcount range and with the plain image
    # bound: identical results; the range adds no blocks (up to round granularity)
    db = synth.gen_db(60_123, 1101)
    q, _ = synth.gen_queries(db, 600, 2101, 0.1, 0.6)
    ref = oracle.knn_brute(db, q, k)
    pop = qd.knn_tree(qd.tree_build(_t(db)), _t(q), k, order=qd.ORDER_BLOCKED, query_stats=True)
    plain = qd.knn_tree(qd.tree_build(_t(db), plain_bound=True), _t(q), k, order=qd.ORDER_BLOCKED, query_stats=True)
    _same(pop, ref)
    _same(plain, ref)
    assert pop[4].cpu().numpy()[:, 0].sum() <= 1.01 * plain[4].cpu().numpy()[:, 0].sum()


def test_blocked_work_counters(qd):
    # while profiling, the search counts its matrix-core tiles and the
    # (query, block) pairs of short lists it ran on the vector ALUs
    db = synth.gen_db(60_123, 1101)
    q, _ = synth.gen_queries(db, 600, 2101, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    qd.profile_enable(True)
    res = qd.knn_tree(tree, _t(q), 10, order=qd.ORDER_BLOCKED, query_stats=True)
    tiles, short = qd.profile_counter("tree_block_tiles"), qd.profile_counter("tree_block_short_pairs")
    qd.profile_enable(False)
    _same(res, oracle.knn_brute(db, q, 10))
    listed = int(res[4].cpu().numpy()[:, 0].astype(np.int64).sum()) - 16 * len(q)  # past round 1
    assert tiles > 0 and short > 0
    assert short <= listed <= short + 256 * tiles
    qd.profile_enable(True)  # counters start again from zero
    assert qd.profile_counter("tree_block_tiles") == 0
    qd.profile_enable(False)


def test_deep_tree_fallback_is_best_first(qd):
    # rows "every bit but bit i" make every split peel off one row (the least
    # popular bit is in all rows but one), so the tree is about 300 levels
    # deep, deeper than the depth-first order's stack; 30,000 all-one rows
    # tie at key 0 for an all-one query, more than a candidate buffer holds,
    # so those queries take the blocked search's fallback, which must then
    # search best-first
    chain = np.full((300, 64), np.uint64(0xFFFFFFFFFFFFFFFF))
    for i in range(300):
        chain[i, i // 64] &= ~(np.uint64(1) << np.uint64(i % 64))
    db = np.concatenate([chain, np.full((30_000, 64), np.uint64(0xFFFFFFFFFFFFFFFF))])
    tree = qd.tree_build(_t(db))
    assert tree.depth > 256
    q = np.concatenate([db[:1], db[150:151], db[-1:], synth.gen_queries(chain, 5, 77, 0.2, 0.5)[0]])
    with pytest.raises(qd.QDError):
        qd.knn_tree(tree, _t(q), 10, order=qd.ORDER_DEPTH_FIRST)  # the stack cannot hold this tree
    for k in (1, 10):
        ref = oracle.knn_brute(db, q, k)
        _same(qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED), ref)
        _same(qd.knn_tree(tree, _t(q), k), ref)
