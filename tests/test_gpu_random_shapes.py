"""Every search path against the oracle on seeded random shapes.

Twelve configurations drawn once from a fixed seed: database sizes from one
row to about 70,000 (ragged against the 8-, 16- and 256-row steps of the
kernels), batches from one query to about 700 (across the 3- and 160-query
switches of the sequential search and the 256-query tiles), k from 1 to 64,
query partiality from 0 to 90% of the source row's bits, and a share of
duplicated rows (ties broken by index).  For each, the sequential search
(automatic path, vector-ALU tile, matrix query tile) and the tree search
(best-first, depth-first, blocked) must equal the oracle's idx, missed,
extra and dist on every query."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _configs():
    rng = np.random.default_rng(20261203)
    out = []
    for i in range(12):
        n = int(rng.choice([1, 2, 7, 31, 257, 4_099, 20_001, 66_667, 70_001]))
        nq = int(rng.choice([1, 2, 3, 5, 16, 17, 159, 160, 161, 300, 700]))
        k = int(rng.choice([1, 2, 5, 10, 33, 64]))
        lo = float(rng.uniform(0.0, 0.5))
        hi = float(min(0.9, lo + rng.uniform(0.0, 0.4)))
        dup = float(rng.choice([0.0, 0.0, 0.1]))
        out.append((i, n, nq, k, lo, hi, dup))
    return out


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda:0")


def _same(res, ref, what):
    idx, missed, extra, dist = (x.cpu().numpy() for x in res[:4])
    assert np.array_equal(idx.view(np.uint32), ref.idx), what
    assert np.array_equal(missed, ref.missed), what
    assert np.array_equal(extra, ref.extra), what
    assert np.array_equal(dist, ref.dist), what


@pytest.mark.parametrize("cfg", _configs(), ids=lambda c: f"n{c[1]}_q{c[2]}_k{c[3]}")
def test_every_path_equals_the_oracle(cfg):
    import paper_2107_03368_amd as qd
    i, n, nq, k, lo, hi, dup = cfg
    db = synth.gen_db(n, 4000 + i)
    if dup and n > 10:
        rng = np.random.default_rng(5000 + i)
        m = int(n * dup)
        db[rng.choice(n, m, replace=False)] = db[rng.choice(n, m, replace=True)]
    q, _ = synth.gen_queries(db, nq, 6000 + i, lo, hi)
    ref = oracle.knn_brute(db, q, k)
    dbt, qt = _t(db), _t(q)
    _same(qd.knn_bruteforce(dbt, qt, k), ref, "sequential, automatic")
    _same(qd.knn_bruteforce(dbt, qt, k, query_tile=16), ref, "sequential, vector-ALU tile")
    _same(qd.knn_bruteforce(dbt, qt, k, query_tile=qd.QUERY_TILE_MATRIX), ref, "sequential, matrix query tile")
    tree = qd.tree_build(dbt)
    for name, order in (("best-first", qd.ORDER_BEST_FIRST), ("depth-first", qd.ORDER_DEPTH_FIRST),
                        ("blocked", qd.ORDER_BLOCKED)):
        _same(qd.knn_tree(tree, qt, k, order=order), ref, name)
