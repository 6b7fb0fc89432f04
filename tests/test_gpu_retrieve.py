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


@pytest.mark.parametrize("use_tree", [False, True])
def test_rows_of_no_object_cast_no_vote(qd, use_tree):
    # a third of the rows carry object ids >= n_obj (some of them the largest
    # uint16): their neighbours cast no vote, on the GPU as in the oracle
    db, obj, off, q, qobj = _workload(20, 200, 6, 15, 60, 63)
    obj = obj.copy()
    obj[::3] = np.where(np.arange(len(obj))[::3] % 2 == 0, 20, 65535).astype(np.uint16)
    for k, threshold in ((1, 3), (5, 10)):
        ref_nn = oracle.knn_brute(db, q, k)
        rv, rw, ru = oracle.votes(ref_nn.idx, obj, 20, off, threshold)
        assert rv.sum() < k * len(q)  # some neighbours did fall on such rows
        tree = qd.tree_build(_t(db)) if use_tree else None
        votes, winner, used = qd.retrieve_objects(_t(q), _t(off), _t(obj), 20, k, threshold, tree=tree,
                                                  db=None if use_tree else _t(db))
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


@pytest.mark.parametrize("path", ["best_first", "best_first_unsplit", "depth_first_split16", "blocked",
                                  "blocked_learned", "sequential", "matrix_cores"])
def test_plan_graph_replays_match_direct_retrieval(qd, path):
    # the matrix-core scan needs >= 65,536 rows and >= 160 descriptors in the
    # largest batch; the plan keeps it for the smaller batches too.  With a
    # model (an untrained one: any model gives exact results), the blocked
    # order's first round starts where the model leads, its descent recorded
    # in the graph on the plan's memory
    import torch
    n_obj = 280 if path == "matrix_cores" else 40
    db, obj, off, q, qobj = _workload(n_obj, 250 if path == "matrix_cores" else 300, 24, 20, 120, 91)
    assert path != "matrix_cores" or (len(db) >= 65_536 and len(q) >= 160)
    use_tree = path not in ("sequential", "matrix_cores")
    order = (qd.ORDER_BLOCKED if path.startswith("blocked") else
             qd.ORDER_DEPTH_FIRST if path.startswith("depth_first") else qd.ORDER_BEST_FIRST)
    # per-query orders: the default split, one wave per query, or 16 subtree searches
    split = {"best_first_unsplit": 1, "depth_first_split16": 16}.get(path, 0)
    model = None
    if path == "blocked_learned":
        model = qd.Model(torch.from_numpy(synth.uniform_f32(qd.MLP_NPARAMS, 3101, -0.05, 0.05)).to("cuda:0"))
    tree = qd.tree_build(_t(db)) if use_tree else None
    dbt = None if use_tree else _t(db)
    plan = qd.Plan(_t(obj), n_obj, max_qdesc=len(q), max_qobj=24, k=5, threshold=10, tree=tree, db=dbt, order=order,
                   query_tile=16 if path == "sequential" else 0, model=model, split=split)
    # batches of different sizes, with eager library work between the replays
    for lo, hi in ((0, 24), (3, 10), (0, 1), (5, 24)):
        sub = np.asarray(off[lo:hi + 1], np.uint64) - off[lo]
        qs = q[int(off[lo]):int(off[hi])]
        got = plan.run(_t(qs), _t(sub))
        ref = qd.retrieve_objects(_t(qs), _t(sub), _t(obj), n_obj, 5, 10, tree=tree, db=dbt, order=order, model=model,
                                  split=split)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        rv, rw, ru = oracle.votes(oracle.knn_brute(db, qs, 5).idx, obj, n_obj, sub, 10)
        assert np.array_equal(got[0].cpu().numpy().view(np.uint32), rv)
        assert np.array_equal(got[1].cpu().numpy(), rw)
        assert np.array_equal(got[2].cpu().numpy().view(np.uint32), ru)


@pytest.mark.parametrize("start", [0, 1, "model"])
def test_blocked_plan_with_several_batches(qd, start):
    # more descriptors than one blocked batch holds (16,384): the plan records
    # two batches, each reading its size from the device; replays of shrinking
    # batches (the second batch empty, then a tiny one) with eager work between;
    # round 1 at the lowest bounds, at the bound's descent, or where a model leads
    import torch
    n_obj, per = 25, 200
    db = synth.gen_db(n_obj * per, 97)
    obj = (np.arange(n_obj * per) // per).astype(np.uint16)
    q, _ = synth.gen_queries(db, 20_000, 98, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    model = None
    if start == "model":
        model = qd.Model(torch.from_numpy(synth.uniform_f32(qd.MLP_NPARAMS, 3102, -0.05, 0.05)).to("cuda:0"))
        start = 0
    plan = qd.Plan(_t(obj), n_obj, max_qdesc=20_000, max_qobj=4, k=10, threshold=10, tree=tree,
                   order=qd.ORDER_BLOCKED, start=start, model=model)
    for nd in (20_000, 16_384, 9, 17_001):
        off = np.array([0, nd // 3, nd // 2, nd], np.uint64)
        got = plan.run(_t(q[:nd]), _t(off))
        ref = qd.retrieve_objects(_t(q[:nd]), _t(off), _t(obj), n_obj, 10, 10, tree=tree, order=qd.ORDER_BLOCKED,
                                  return_nn=True, model=model)
        torch.cuda.synchronize()
        for a, b in zip(got, ref[:3]):
            assert torch.equal(a, b)
        nn = ref[3].cpu().numpy().view(np.uint32)
        rows = np.array([0, nd // 2, nd - 1])
        assert np.array_equal(nn[rows], oracle.knn_brute(db, q[rows], 10).idx)
        rv, rw, ru = oracle.votes(nn, obj, n_obj, off, 10)
        assert np.array_equal(got[0].cpu().numpy().view(np.uint32), rv)


def test_autotuner_returns_a_timed_exact_configuration(qd):
    db = synth.gen_db(50_000, 95)
    q, _ = synth.gen_queries(db, 300, 96, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    ref = oracle.knn_brute(db, q[:4], 10)
    for kw in (dict(tree=tree), dict(db=_t(db))):
        best, cands = qd.autotune(_t(q), 10, reps=2, **kw)
        assert len(cands) >= 3 and all(c["ms"] > 0 for c in cands)
        assert best["ms"] == min(c["ms"] for c in cands)
        if "tree" in kw:
            assert any(c["order"] == qd.ORDER_BLOCKED for c in cands)  # the round schedules were timed
            assert len({c["schedule"] for c in cands if c["order"] == qd.ORDER_BLOCKED}) >= 5
            res = qd.knn_tree(tree, _t(q), 10, order=best["order"], waves_per_cu=best["waves_per_cu"],
                              schedule=best["schedule"], start=best["start"])
        else:
            res = qd.knn_bruteforce(_t(db), _t(q), 10, query_tile=best["query_tile"])
        assert np.array_equal(res[0].cpu().numpy().view(np.uint32)[:4], ref.idx)


def _prefix_votes(nn_idx, obj, n_obj, off, used):
    """Oracle histogram over the first used[g] descriptors of each object."""
    out = np.zeros((len(off) - 1, n_obj), np.uint32)
    for g in range(len(off) - 1):
        rows = nn_idx[int(off[g]):int(off[g]) + int(used[g])].reshape(-1)
        o = obj[rows[rows != 0xFFFFFFFF]].astype(np.int64)
        np.add.at(out[g], o[o < n_obj], 1)
    return out


@pytest.mark.parametrize("order", ["brute", "best_first", "blocked"])
@pytest.mark.parametrize("k,threshold", [(1, 10), (5, 10), (3, 1), (2, 255)])
def test_early_exit_matches_full_retrieval(qd, order, k, threshold):
    # query objects of 15-300 descriptors: several rounds (16, 32, 64, ...)
    db, obj, off, q, qobj = _workload(40, 300, 9, 15, 300, 91)
    ref_nn = oracle.knn_brute(db, q, k)
    rv, rw, ru = oracle.votes(ref_nn.idx, obj, 40, off, threshold)
    tree = None if order == "brute" else qd.tree_build(_t(db))
    o = qd.ORDER_BLOCKED if order == "blocked" else qd.ORDER_BEST_FIRST
    votes, winner, used, searched = qd.retrieve_objects_early(_t(q), _t(off), _t(obj), 40, k, threshold, tree=tree,
                                                              db=_t(db) if tree is None else None, order=o)
    assert np.array_equal(winner.cpu().numpy(), rw)
    assert np.array_equal(used.cpu().numpy().view(np.uint32), ru)
    assert np.array_equal(votes.cpu().numpy().view(np.uint32), _prefix_votes(ref_nn.idx, obj, 40, off, ru))
    assert int(ru.sum()) <= searched <= len(q)


def test_early_exit_searches_a_fraction_at_scale(qd):
    # 300 objects x 5,000 descriptors, 128 query objects of 200-4,000 descriptors, k = 5,
    # threshold 10: the decisions equal the full retrieval's with far fewer searches
    db, obj, off, q, qobj = _workload(300, 5000, 128, 200, 4000, 1002)
    tree = qd.tree_build(_t(db))
    full = qd.retrieve_objects(_t(q), _t(off), _t(obj), 300, 5, 10, tree=tree, order=qd.ORDER_BLOCKED)
    votes, winner, used, searched = qd.retrieve_objects_early(_t(q), _t(off), _t(obj), 300, 5, 10, tree=tree,
                                                              order=qd.ORDER_BLOCKED)
    assert np.array_equal(winner.cpu().numpy(), full[1].cpu().numpy())
    assert np.array_equal(used.cpu().numpy(), full[2].cpu().numpy())
    print(f"searched {searched} of {len(q)} descriptors")
    assert searched < 0.1 * len(q)
