"""Bit-plane sequential search against the CPU oracle and the row scan.

Results must equal the oracle's sequential search bit for bit: ragged row
counts (partial last plane words and blocks of eight words), single queries
and batches, k up to 64, queries with no bits and with every bit (the widest
counters), many rows tied at one key, and 1M rows."""
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


@pytest.mark.parametrize("k", [1, 10, 64])
def test_planes_match_oracle_10k(qd, small_db, small_queries, k):
    q, _ = small_queries
    pl = qd.Planes(_t(small_db))
    _same(qd.knn_planes(pl, _t(q), k), oracle.knn_brute(small_db, q, k))
    _same(qd.knn_planes(pl, _t(q[:1]), k), oracle.knn_brute(small_db, q[:1], k))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 511, 513, 4097, 10_007])
def test_planes_ragged_sizes(qd, n):
    db = synth.gen_db(n, 4100 + n)
    q, _ = synth.gen_queries(db, 7, 4200 + n, 0.1, 0.6)
    pl = qd.Planes(_t(db))
    for k in (1, 5, 64):
        _same(qd.knn_planes(pl, _t(q), k), oracle.knn_brute(db, q, k))


def test_planes_degenerate_queries_and_ties(qd):
    base = synth.gen_db(3000, 4301)
    db = np.concatenate([base, np.repeat(base[7:8], 500, axis=0), np.zeros((40, 64), np.uint64),
                         np.full((3, 64), np.uint64(0xFFFFFFFFFFFFFFFF))])
    q = np.concatenate([np.zeros((1, 64), np.uint64), np.full((1, 64), np.uint64(0xFFFFFFFFFFFFFFFF)),
                        base[7:8], synth.gen_queries(base, 5, 4302, 0.2, 0.6)[0]])
    pl = qd.Planes(_t(db))
    for k in (1, 10, 64):
        _same(qd.knn_planes(pl, _t(q), k), oracle.knn_brute(db, q, k))


def test_planes_1m(qd):
    db = synth.gen_db(1_000_000, 1001)
    q, _ = synth.gen_queries(db, 40, 2001, 0.1, 0.6)
    pl = qd.Planes(_t(db))
    for k in (1, 10):
        res = qd.knn_planes(pl, _t(q), k)
        for a, b in zip(_np(res), _np(qd.knn_bruteforce(_t(db), _t(q), k))):
            assert np.array_equal(a, b)
        rows = np.array([0, 17, 39])
        _same(res, oracle.knn_brute(db, q[rows], k), rows)


def test_planes_argument_errors(qd):
    import torch
    db = synth.gen_db(100, 4401)
    pl = qd.Planes(_t(db))
    q = _t(db[:2])
    with pytest.raises(qd.QDError):
        qd.knn_planes(pl, q, 0)
    with pytest.raises(qd.QDError):
        qd.knn_planes(pl, q, 65)
    assert qd.knn_planes(pl, torch.zeros((0, 64), dtype=torch.int64, device="cuda:0"), 3)[0].shape == (0, 3)
