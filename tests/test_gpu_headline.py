"""Every search path at the headline shape: 10,000,000 database rows, 8,192
partial noisy queries (10-60% of the set bits cleared, 8 bits flipped),
k = 10, in the launch configuration the benchmark times.  Sequential search
(matrix cores), tree search best-first, depth-first, blocked, and depth-first
in a learned order must return the same idx, missed, extra and dist for
every query, and equal the oracle's sequential search on 32 queries sampled
across the batch."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_all_paths_at_10m_x_8192():
    import torch
    import paper_2107_03368_amd as qd
    from oracle import mlp as omlp
    dev = "cuda:0"
    n, nq, k = 10_000_000, 8192, 10
    db = synth.gen_db(n, 1003)
    q, _ = synth.gen_queries(db, nq, 2003, 0.1, 0.6)
    dbt = torch.from_numpy(db.view(np.int64)).to(dev)
    qt = torch.from_numpy(q.view(np.int64)).to(dev)
    print(f"10M x 8,192: brute", flush=True)
    ref = [x.cpu().numpy() for x in qd.knn_bruteforce(dbt, qt, k)]
    tree = qd.tree_build(dbt)
    model = qd.Model(torch.from_numpy(synth.uniform_f32(omlp.NPARAMS, 3003, -0.05, 0.05)).to(dev))
    scores = qd.model_score_tree(model, tree, qt, 2047)
    paths = {
        "best_first": lambda: qd.knn_tree(tree, qt, k),
        "depth_first": lambda: qd.knn_tree(tree, qt, k, order=qd.ORDER_DEPTH_FIRST),
        "blocked": lambda: qd.knn_tree(tree, qt, k, order=qd.ORDER_BLOCKED),
        "learned": lambda: qd.knn_tree(tree, qt, k, order=qd.ORDER_DEPTH_FIRST, scores=scores),
    }
    for name, fn in paths.items():
        print(f"10M x 8,192: {name}", flush=True)
        out = [x.cpu().numpy() for x in fn()[:4]]
        for a, b, what in zip(out, ref, ("idx", "missed", "extra", "dist")):
            assert np.array_equal(a, b), (name, what, int((a != b).any(1).sum()))
    rows = np.arange(0, nq, nq // 32) + np.arange(32) * 7  # 32 queries spread over the batch
    print(f"10M x 8,192: oracle on {len(rows)} queries", flush=True)
    o = oracle.knn_brute(db, q[rows], k)
    assert np.array_equal(ref[0][rows].view(np.uint32), o.idx)
    assert np.array_equal(ref[1][rows], o.missed)
    assert np.array_equal(ref[2][rows], o.extra)
    assert np.array_equal(ref[3][rows], o.dist)
