"""GPU frontier-order model (BF16 MFMA kernels, FP32 accumulation) against the
float64 CPU oracle: features, forward scores, gradients; plus training,
traces and the exactness of the learned-order search."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qd():
    import paper_2107_03368_amd as qd
    return qd


def _t(a):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to("cuda:0")


@pytest.fixture(scope="module")
def setup(qd, small_db, small_queries):
    q, _ = small_queries
    tree = qd.tree_build(_t(small_db))
    ex = tree.export()
    parent = np.full(tree.n_nodes, -1, np.int64)
    depth = np.zeros(tree.n_nodes, np.int64)
    for i in range(tree.n_nodes):
        if ex["child"][i, 0] >= 0:
            parent[ex["child"][i]] = i
            depth[ex["child"][i]] = depth[i] + 1
    return q, tree, ex, parent, depth


def _pairs(n_nodes, nq, per, seed):
    rng = np.random.default_rng(seed)
    pq = np.repeat(np.arange(nq, dtype=np.uint32), per)
    pn = rng.integers(0, n_nodes, nq * per).astype(np.uint32)
    pn[0] = 0  # the root
    return pq, pn


def test_features_match_oracle(qd, setup):
    q, tree, ex, parent, depth = setup
    pq, pn = _pairs(tree.n_nodes, 10, 13, 1)
    f = qd.model_features(tree, _t(q), _t(pq), _t(pn)).cpu().numpy()
    ref = omlp.features(q, ex["or_img"], ex["child"], parent, depth, ex["count"], pq, pn)
    assert np.allclose(f, ref, rtol=1e-6, atol=1e-6)


def _params(seed):
    return synth.uniform_f32(omlp.NPARAMS, seed, -0.05, 0.05)


@pytest.mark.parametrize("nq,per", [(7, 19), (40, 64)])
def test_forward_matches_oracle(qd, setup, nq, per):
    q, tree, *_ = setup
    params = _params(5)
    model = qd.Model(_t(params))
    pq, pn = _pairs(tree.n_nodes, nq, per, 2)
    feat = qd.model_features(tree, _t(q), _t(pq), _t(pn))
    s = qd.model_forward(model, _t(q), _t(pq), feat).cpu().numpy()
    ref, _ = omlp.forward(params, q, pq, feat.cpu().numpy())
    assert np.abs(s - ref).max() <= 1e-2 * (np.abs(ref).max() + 1e-3)
    assert np.corrcoef(s, ref)[0, 1] > 0.999


def test_gradients_match_oracle_and_are_reproducible(qd, setup):
    import torch
    q, tree, *_ = setup
    params = _params(7)
    model = qd.Model(_t(params))
    nq, per = 12, 37
    pq, pn = _pairs(tree.n_nodes, nq, per, 3)
    qoff = np.arange(0, nq * per + 1, per, dtype=np.int64)
    labels = (np.random.default_rng(4).random(nq * per) < 0.3).astype(np.float32)
    feat = qd.model_features(tree, _t(q), _t(pq), _t(pn))
    g, loss = qd.model_gradients(model, _t(q[:nq]), _t(qoff), _t(pq), feat, _t(labels))
    g2, _ = qd.model_gradients(model, _t(q[:nq]), _t(qoff), _t(pq), feat, _t(labels))
    assert torch.equal(g, g2)
    g = g.cpu().numpy().astype(np.float64)
    rloss, rg = omlp.loss_and_grad(params, q[:nq], pq, feat.cpu().numpy(), labels)
    assert abs(loss.item() - rloss) <= 1e-3 * abs(rloss)
    o = 0
    for name, shape in omlp.SIZES:
        n = int(np.prod(shape))
        a, b = g[o:o + n], rg[o:o + n]
        o += n
        if np.linalg.norm(b) == 0:
            assert np.linalg.norm(a) <= 1e-6
            continue
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), name
        assert a @ b / (np.linalg.norm(a) * np.linalg.norm(b)) >= 0.999, name
        # element by element: every entry within 1% of the block's largest
        # oracle entry (bf16 operands carry 2^-8 relative rounding; a wrong
        # entry hidden in a long block's norm fails here)
        err = np.abs(a - b).max()
        assert err <= 1e-2 * np.abs(b).max(), (name, err / np.abs(b).max(), int(np.abs(a - b).argmax()))


def test_trace_pairs_follow_the_search(qd, setup):
    q, tree, ex, parent, _ = setup
    n_traced = min(255, tree.n_nodes)
    idx, missed, extra, dist, vis = qd.knn_tree_traced(tree, _t(q), 10, n_traced)
    pq, pn, lab, qoff = qd.trace_pairs(tree, idx, vis, n_traced)
    vis = vis.cpu().numpy().view(np.uint32)
    pq, pn, lab, qoff = pq.cpu().numpy(), pn.cpu().numpy(), lab.cpu().numpy(), qoff.cpu().numpy()
    idx = idx.cpu().numpy().view(np.uint32)
    iperm = np.empty_like(ex["perm"])
    iperm[ex["perm"]] = np.arange(len(iperm), dtype=np.uint32)
    assert qoff[0] == 0 and qoff[-1] == len(pq)
    for j in range(len(q)):
        visited = {n for n in range(n_traced) if (vis[j, n // 32] >> (n % 32)) & 1}
        expect = [n for n in range(1, n_traced) if parent[n] in visited]
        got = pn[qoff[j]:qoff[j + 1]]
        assert list(got) == expect and (pq[qoff[j]:qoff[j + 1]] == j).all()
        pos = iperm[idx[j]]
        for n, l in zip(got, lab[qoff[j]:qoff[j + 1]]):
            b, c = ex["begin"][n], ex["count"][n]
            assert l == float(((pos >= b) & (pos < b + c)).any())


def test_training_lowers_the_loss_and_the_learned_search_is_exact(qd, setup, small_db):
    import torch
    q, tree, *_ = setup
    model = qd.Model(_t(_params(11)))
    n_traced = min(511, tree.n_nodes)
    losses, npairs = qd.model_train(model, tree, _t(q), 10, n_traced, epochs=8, batch_queries=10, lr=2e-3)
    assert npairs > 0
    first, last = np.nanmean(losses[:10]), np.nanmean(losses[-10:])
    assert last < first
    scores = qd.model_score_tree(model, tree, _t(q), n_traced)
    # scores equal the forward pass over the same explicit pairs
    pq = np.repeat(np.arange(len(q), dtype=np.uint32), n_traced)
    pn = np.tile(np.arange(n_traced, dtype=np.uint32), len(q))
    feat = qd.model_features(tree, _t(q), _t(pq), _t(pn))
    s2 = qd.model_forward(model, _t(q), _t(pq), feat).reshape(len(q), n_traced)
    assert torch.equal(scores, s2)
    for k in (1, 10):
        ref = oracle.knn_brute(small_db, q, k)
        res = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_DEPTH_FIRST, scores=scores)
        assert np.array_equal(res[0].cpu().numpy().view(np.uint32), ref.idx)
        assert np.array_equal(res[1].cpu().numpy(), ref.missed)
        assert np.array_equal(res[2].cpu().numpy(), ref.extra)
        assert np.array_equal(res[3].cpu().numpy(), ref.dist)


def test_trained_order_gain_over_bound_order(qd):
    """What the trained network gains: a model trained on traces of the exact
    search over a 1M-row database orders the depth-first frontier of a
    different 1M-row database; it must visit fewer nodes than the bound
    order, and its results stay exact."""
    import torch
    dev = "cuda:0"
    tdb = synth.gen_db(1_000_000, 1001)
    ttree = qd.tree_build(torch.from_numpy(tdb.view(np.int64)).to(dev))
    tq, _ = synth.gen_queries(tdb, 4096, 2001, 0.1, 0.6)
    model = qd.Model(_t(synth.uniform_f32(omlp.NPARAMS, 3003, -0.05, 0.05)))
    nb = 4096 // 32
    qd.model_train(model, ttree, _t(tq), 10, 2047, 8, 32, 2e-3, batch_order=synth.permutation(nb, 3004))
    db = synth.gen_db(1_000_000, 1005)
    q, _ = synth.gen_queries(db, 1024, 2005, 0.1, 0.6)
    tree = qd.tree_build(_t(db))
    qt = _t(q)
    # one wave per query, so the node counts do not depend on timing
    plain = qd.knn_tree(tree, qt, 10, order=qd.ORDER_DEPTH_FIRST, totals=True, split=1)
    scores = qd.model_score_tree(model, tree, qt, 2047)
    learned = qd.knn_tree(tree, qt, 10, order=qd.ORDER_DEPTH_FIRST, scores=scores, totals=True, split=1)
    best = qd.knn_tree(tree, qt, 10, totals=True, split=1)
    for a, b in zip(plain[:4], learned[:4]):
        assert torch.equal(a, b)
    n_plain, n_learned, n_best = (r[-1]["nodes_visited"] / len(q) for r in (plain, learned, best))
    print(f"nodes visited per query: bound order {n_plain:.0f}, learned order {n_learned:.0f}, "
          f"best-first {n_best:.0f}")
    assert n_best <= n_learned < n_plain


def test_model_handle_orders_depth_first_as_explicit_scores(qd, setup):
    # a model passed with the search scores the same nodes the caller would
    # score with qd_model_score_tree: same results, same work per query
    q, tree, *_ = setup
    model = qd.Model(_t(_params(13)))
    n = min(511, tree.n_nodes)
    sc = qd.model_score_tree(model, tree, _t(q), n)
    a = qd.knn_tree(tree, _t(q), 10, order=qd.ORDER_DEPTH_FIRST, scores=sc, query_stats=True, split=1)
    b = qd.knn_tree(tree, _t(q), 10, order=qd.ORDER_DEPTH_FIRST, model=model, n_scored=n, query_stats=True, split=1)
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    with pytest.raises(qd.QDError):
        qd.knn_tree(tree, _t(q), 10, model=model)  # best-first takes no model


@pytest.fixture(scope="module")
def blocked_case(qd):
    # 60,123 rows (235 blocks, the last ragged), 600 queries: several rounds and tiles
    db = synth.gen_db(60_123, 1101)
    q, _ = synth.gen_queries(db, 600, 2101, 0.1, 0.6)
    return db, q, qd.tree_build(_t(db))


@pytest.mark.parametrize("k,schedule", [(1, (0, 0, 0)), (10, (0, 0, 0)), (10, (4, 0, 2)), (50, (64, 0, 2)),
                                        (64, (1, 100_000, 2))])
def test_learned_start_of_the_blocked_search_is_exact(qd, blocked_case, k, schedule):
    # round 1 where the model leads (an untrained model: an arbitrary start);
    # the last case overflows the candidate buffers in round 2, so queries
    # repeat it with their round-1 blocks still marked done
    db, q, tree = blocked_case
    model = qd.Model(_t(_params(17)))
    ref = oracle.knn_brute(db, q, k)
    res = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, model=model, schedule=schedule, query_stats=True)
    out = [x.cpu().numpy() for x in res]
    assert np.array_equal(out[0].view(np.uint32), ref.idx)
    assert np.array_equal(out[1], ref.missed) and np.array_equal(out[2], ref.extra)
    assert np.array_equal(out[3], ref.dist)
    plain = qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, schedule=schedule, query_stats=True)
    # the learned start changed the work of some queries (the path ran), not the results
    assert (plain[4].cpu().numpy() != out[4]).any()


def test_learned_start_with_the_per_query_fallback(qd):
    # 30,000 copies of one row: round 2 overflows for good and the queries are
    # searched again best-first, after a learned round 1
    rng_db = synth.gen_db(4000, 75)
    db = np.concatenate([rng_db, np.repeat(rng_db[:1], 30_000, axis=0)])
    q = np.concatenate([rng_db[:3], synth.gen_queries(rng_db, 5, 76, 0.2, 0.5)[0]])
    tree = qd.tree_build(_t(db))
    model = qd.Model(_t(_params(19)))
    for k in (1, 10):
        ref = oracle.knn_brute(db, q, k)
        out = [x.cpu().numpy() for x in qd.knn_tree(tree, _t(q), k, order=qd.ORDER_BLOCKED, model=model)]
        assert np.array_equal(out[0].view(np.uint32), ref.idx)
        assert np.array_equal(out[1], ref.missed) and np.array_equal(out[2], ref.extra)
        assert np.array_equal(out[3], ref.dist)
