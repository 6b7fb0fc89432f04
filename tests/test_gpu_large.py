"""Sequential and blocked tree search on a database larger than one dispatch
of one workgroup per tile can cover: 34M rows x 16,384 queries is 8.7M
matrix-core tiles, more than 2^32 work-items at 512 per workgroup, so the
kernels must loop over tiles.  Sampled queries whose neighbours lie beyond
row 2^24 are checked against the oracle, and the two GPU paths against each
other on every query."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_search_beyond_one_dispatch():
    import torch
    import paper_2107_03368_amd as qd
    n, nq, k = 34_000_000, 16_384, 10
    db = synth.gen_db(n, 1106)
    src = np.concatenate([np.arange(33_000_000, 33_000_000 + nq // 2, dtype=np.uint32),
                          np.arange(0, nq - nq // 2, dtype=np.uint32)])
    q, _ = synth.gen_queries(db, nq, 2106, 0.1, 0.5, src=src)
    dbt = torch.from_numpy(db.view(np.int64)).to("cuda:0")
    qt = torch.from_numpy(q.view(np.int64)).to("cuda:0")
    brute = [x.cpu().numpy() for x in qd.knn_bruteforce(dbt, qt, k)]
    tree = qd.tree_build(dbt)
    blocked = [x.cpu().numpy() for x in qd.knn_tree(tree, qt, k, order=qd.ORDER_BLOCKED)]
    for a, b in zip(brute, blocked):
        assert np.array_equal(a, b)
    rows = np.array([0, 1, nq // 2 - 1, nq // 2, nq - 1])
    ref = oracle.knn_brute(db, q[rows], k)
    assert np.array_equal(brute[0][rows].view(np.uint32), ref.idx)
    assert np.array_equal(brute[3][rows], ref.dist)
    assert (ref.idx[:2, 0] >= 1 << 24).all()  # the nearest rows lie beyond 2^24
