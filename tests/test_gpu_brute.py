"""GPU sequential-search k-NN against the CPU oracle, through the C ABI.

Bit-exact on idx, missed, extra and dist (the float is the same correctly
rounded double quotient on both sides)."""
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
    idx, missed, extra, dist = (x.cpu().numpy() for x in res)
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



@pytest.mark.parametrize("k", [1, 10])
def test_small_workload_matches_oracle(qd, small_db, small_queries, k):
    q, _ = small_queries
    ref = oracle.knn_brute(small_db, q, k)
    _same(qd.knn_bruteforce(_t(small_db), _t(q), k), ref)


@pytest.mark.parametrize("tile,parts", [(1, 1), (2, 3), (4, 7), (8, 64), (16, 4096), (16, 1), (1, 4096)])
def test_result_independent_of_launch_shape(qd, small_db, small_queries, tile, parts):
    q, _ = small_queries
    q = q[:37]  # ragged against every query tile
    db = small_db[:9_999]  # ragged against the 8-row step
    ref = oracle.knn_brute(db, q, 13)
    _same(qd.knn_bruteforce(_t(db), _t(q), 13, query_tile=tile, row_parts=parts), ref)


@pytest.mark.parametrize("parts", [0, 1, 5, 4096])
def test_matrix_query_tile_independent_of_launch_shape(qd, small_db, small_queries, parts):
    # tiles of 16 queries on the matrix cores: 37 queries (ragged against the
    # tile) over 9,999 rows (ragged against the 16-row product)
    q, _ = small_queries
    q, db = q[:37], small_db[:9_999]
    ref = oracle.knn_brute(db, q, 13)
    _same(qd.knn_bruteforce(_t(db), _t(q), 13, query_tile=qd.QUERY_TILE_MATRIX, row_parts=parts), ref)


def test_ties_duplicates_and_degenerate_queries(qd):
    rng = np.random.default_rng(3)
    base = synth.gen_db(200, 51)
    db = np.concatenate([base, base[:50], base[:50], np.zeros((7, 64), np.uint64),
                         np.full((3, 64), np.uint64(0xFFFFFFFFFFFFFFFF))])
    db = db[rng.permutation(len(db))]
    q = np.concatenate([base[:20], np.zeros((2, 64), np.uint64), np.full((2, 64), np.uint64(0xFFFFFFFFFFFFFFFF)),
                        synth.gen_queries(base, 10, 52, 0.3, 0.6)[0]])
    for k in (1, 5, 64):
        ref = oracle.knn_brute(db, q, k)
        _same(qd.knn_bruteforce(_t(db), _t(q), k), ref)


def test_fewer_rows_than_k_and_single_row(qd, small_db, small_queries):
    q, _ = small_queries
    for n, k in ((3, 5), (1, 1), (1, 64), (63, 64)):
        ref = oracle.knn_brute(small_db[:n], q[:9], k)
        _same(qd.knn_bruteforce(_t(small_db[:n]), _t(q[:9]), k), ref)


def test_popcount_rows(qd, small_db):
    pop = qd.popcount_rows(_t(small_db)).cpu().numpy().astype(np.int64)
    ref = np.unpackbits(small_db.view(np.uint8), axis=1).sum(1)
    assert np.array_equal(pop, ref)


@pytest.fixture(scope="module")
def db_1m():
    return synth.gen_db(1_000_000, 1001)


@pytest.mark.parametrize("k", [1, 10, 50])
def test_1m_workload_sampled_queries(qd, db_1m, k):
    # the full 4,096-query batch runs on the GPU in the launch shape the
    # benchmark uses; the oracle scores a sample of the queries
    q, _ = synth.gen_queries(db_1m, 4096, 2001, 0.1, 0.6)
    res = qd.knn_bruteforce(_t(db_1m), _t(q), k)
    rows = _sample([0, 1, 777, 2048, 4095], 4096, 31)
    ref = oracle.knn_brute(db_1m, q[rows], k)
    _same(res, ref, rows)


def _degenerate_rows(n, seed):
    """n rows: all zero, all one, and dense random rows (about half the bits)."""
    rng = np.random.default_rng(seed)
    dense = rng.integers(0, 2 ** 63, (n, 64), dtype=np.int64).view(np.uint64) ^ \
        (rng.integers(0, 2, (n, 64), dtype=np.uint64) << np.uint64(63))
    dense[0::3] = 0
    dense[1::3] = np.uint64(0xFFFFFFFFFFFFFFFF)
    return dense


@pytest.mark.parametrize("nq", [600, 161])
def test_matrix_core_path_equals_register_scan_and_oracle(qd, nq):
    # >= 160 queries over >= 65,536 rows take the FP4 matrix-core path by
    # default; the register-tiled scan (an explicit query tile) must agree bit
    # for bit, and the oracle on every query.  Among them: all-zero and all-one
    # queries (|q| = 0 and 4096, the ends of the weights) and all-zero,
    # all-one and dense rows (overlap counts up to 4096)
    db = synth.gen_db(100_003, 1011)  # ragged against the 256-row tile
    db[5000:5030] = _degenerate_rows(30, 1013)
    q, _ = synth.gen_queries(db, nq, 2011, 0.1, 0.6)  # ragged against the 256-query tile
    q[100:120] = 0
    q[130:150] = np.uint64(0xFFFFFFFFFFFFFFFF)
    q[nq - 10:nq - 4] = _degenerate_rows(6, 1014)
    for k in (1, 10, 50):
        a = qd.knn_bruteforce(_t(db), _t(q), k)
        b = qd.knn_bruteforce(_t(db), _t(q), k, query_tile=16)
        for x, y in zip(a, b):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
        _same(a, oracle.knn_brute(db, q, k))


@pytest.mark.parametrize("nq", [1, 3, 4, 15, 16, 17, 40])
def test_matrix_query_tile_batch_sizes_and_degenerate_inputs(qd, nq):
    # small batches (3 or more queries take the matrix query tile by default):
    # every batch size around the 16-query tile, all-zero, all-one and dense
    # rows and queries (|q| = 0 and 4096, overlap counts up to 4096), k up to
    # the 64-entry limit; equal to the oracle and to the vector-ALU scan
    db = synth.gen_db(20_011, 1021)
    db[777:807] = _degenerate_rows(30, 1022)
    q, _ = synth.gen_queries(db, nq, 2021, 0.1, 0.6)
    if nq >= 3:
        q[:3] = _degenerate_rows(3, 1023)
    for k in (1, 10, 64):
        a = qd.knn_bruteforce(_t(db), _t(q), k, query_tile=qd.QUERY_TILE_MATRIX)
        b = qd.knn_bruteforce(_t(db), _t(q), k, query_tile=16)
        for x, y in zip(a, b):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
        _same(a, oracle.knn_brute(db, q, k))
        if nq >= 3:
            _same(qd.knn_bruteforce(_t(db), _t(q), k), oracle.knn_brute(db, q, k))


def test_matrix_core_path_overflow_falls_back_exactly(qd):
    # the sample rows (the first rows) hold only the image corners, which no ring
    # arc reaches: every query misses all of its bits there and pays for ~900
    # extra bits, so the sample's k-th key admits nearly every other row; every
    # query overflows its candidate buffer and is searched again by the
    # register-tiled scan
    db = synth.gen_db(70_000, 1012)
    rr, cc = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    corner = ((rr - 31.5) ** 2 + (cc - 31.5) ** 2 > 32.5 ** 2)
    db[:8000] = synth.from_bits(1, [list(np.flatnonzero(corner.reshape(-1)))])[0]
    q, _ = synth.gen_queries(db[8000:], 520, 2012, 0.1, 0.6)
    a = qd.knn_bruteforce(_t(db), _t(q), 10)
    b = qd.knn_bruteforce(_t(db), _t(q), 10, query_tile=16)
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    rows = np.array([0, 519])
    _same(a, oracle.knn_brute(db, q[rows], 10), rows)
