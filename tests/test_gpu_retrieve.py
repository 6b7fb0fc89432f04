"""GPU retrieval by voting against the CPU oracle (Section 3's pipeline)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qd():
    import paper_2107_03368_amd as qd
    return qd


def _t(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to("cuda:0")


def _workload(n_obj, per, nqo, mmin, mmax, seed):
    db = synth.gen_db(n_obj * per, seed)
    obj = (np.arange(n_obj * per) // per).astype(np.uint16)
    off, rows, qobj = synth.gen_query_objects(n_obj, per, nqo, seed + 1, mmin, mmax)
    q, _ = synth.gen_queries(db, len(rows), seed + 2, 0.2, 0.7, src=rows)
    return db, obj, off, q, qobj


@pytest.mark.parametrize("use_tree", [False, True])
@pytest.mark.parametrize("k,threshold", [(1, 10), (5, 10), (3, 1), (2, 255)])
def test_votes_match_oracle(qd, use_tree, k, threshold):
    db, obj, off, q, qobj = _workload(20, 200, 6, 15, 60, 61)
    ref_nn = oracle.knn_brute(db, q, k)
    rv, rw, ru = oracle.votes(ref_nn.idx, obj, 20, off, threshold)
    tree = qd.tree_build(_t(db)) if use_tree else None
    votes, winner, used, nn = qd.retrieve_objects(_t(q), _t(off), _t(obj), 20, k, threshold, tree=tree,
                                                  db=None if use_tree else _t(db), return_nn=True)
    assert np.array_equal(nn.cpu().numpy().view(np.uint32), ref_nn.idx)
    assert np.array_equal(votes.cpu().numpy().view(np.uint32), rv)
    assert np.array_equal(winner.cpu().numpy(), rw)
    assert np.array_equal(used.cpu().numpy().view(np.uint32), ru)


def test_many_objects_and_empty_query_objects(qd):
    # more objects than the LDS histogram holds; some query objects have no descriptors
    n_obj, per = 9000, 2
    db = synth.gen_db(n_obj * per, 81)
    obj = (np.arange(n_obj * per) // per).astype(np.uint16)
    rows = np.array([5, 6, 7, 1000, 1001, 17999], np.uint32)
    q, _ = synth.gen_queries(db, len(rows), 82, 0.0, 0.0, nflip=0, src=rows)
    off = np.array([0, 3, 3, 6, 6], np.uint64)
    ref = oracle.knn_brute(db, q, 2)
    rv, rw, ru = oracle.votes(ref.idx, obj, n_obj, off, 2)
    votes, winner, used = qd.retrieve_objects(_t(q), _t(off), _t(obj), n_obj, 2, 2, db=_t(db))
    assert np.array_equal(votes.cpu().numpy().view(np.uint32), rv)
    assert np.array_equal(winner.cpu().numpy(), rw)
    assert np.array_equal(used.cpu().numpy().view(np.uint32), ru)


def test_objects_workload_full_scale(qd):
    # 300 objects x 5,000 descriptors, 128 query objects of 200-4,000 descriptors, k = 5:
    # the votes of the whole batch follow the oracle's vote rule on the GPU's neighbours,
    # and sampled descriptors' neighbours match the oracle's sequential search
    db, obj, off, q, qobj = _workload(300, 5000, 128, 200, 4000, 1002)
    tree = qd.tree_build(_t(db))
    votes, winner, used, nn = qd.retrieve_objects(_t(q), _t(off), _t(obj), 300, 5, 10, tree=tree, return_nn=True)
    nn = nn.cpu().numpy().view(np.uint32)
    rv, rw, ru = oracle.votes(nn, obj, 300, off, 10)
    assert np.array_equal(votes.cpu().numpy().view(np.uint32), rv)
    assert np.array_equal(winner.cpu().numpy(), rw)
    assert np.array_equal(used.cpu().numpy().view(np.uint32), ru)
    rows = np.array([0, 1, 12345, len(q) // 2, len(q) - 1])
    assert np.array_equal(nn[rows], oracle.knn_brute(db, q[rows], 5).idx)
    assert (rw == qobj).mean() >= 0.95  # the workload is retrievable
