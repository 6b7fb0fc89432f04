"""Object-level distance scores on the GPU against the CPU oracle.

Every score must equal the oracle's bit for bit: the per-object minima are
exact integers and both sides add the float64 terms in descriptor order.
Cases span several row tiles per object with ragged ends, objects without
rows, rows of no object, several descriptor tiles, empty query objects,
several descriptor batches (65,536 objects) and the retrieval workload's
size (sampled query objects)."""
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
    if dtype is not None:
        a = a.view(dtype)
    elif a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to("cuda:0")


def _gpu(qd, db, obj, n_obj, q, qoff):
    return qd.object_scores(_t(db), _t(obj, np.int16), n_obj, _t(q), _t(qoff, np.int64)).cpu().numpy()


def _objects(sizes, seed, extra_none=0):
    """Rows of objects with the given row counts, interleaved, plus rows of no object."""
    n = int(sum(sizes)) + extra_none
    db = synth.gen_db(n, seed)
    parts = [np.full(c, o, np.uint16) for o, c in enumerate(sizes)]
    if extra_none:
        parts.append(np.full(extra_none, len(sizes) + 3, np.uint16))
    obj = np.concatenate(parts)
    p = synth.permutation(n, seed + 1)
    return db, obj[p]


def _query_objects(db, obj, n_obj, sizes, seed):
    """Query objects of the given descriptor counts, each from one object's rows."""
    rng_src = synth.permutation(len(db), seed)
    src, off = [], [0]
    for g, m in enumerate(sizes):
        o = g % n_obj
        rows = [r for r in rng_src if obj[r] == o][:m]
        if len(rows) < m:
            rows = list(rng_src[:m])
        src += rows
        off.append(off[-1] + m)
    q, _ = synth.gen_queries(db, len(src), seed + 1, 0.1, 0.6, src=np.array(src, np.uint32))
    return q, np.array(off, np.uint64)


def test_scores_match_oracle_small(qd):
    # 14 objects: several tiles per object, ragged ends, one of 1 row, two empty
    sizes = [700, 256, 257, 1, 0, 513, 90, 300, 0, 1024, 45, 600, 255, 380]
    db, obj = _objects(sizes, 3101, extra_none=77)
    n_obj = len(sizes)
    # 611 descriptors (three tiles, the last ragged) in 9 query objects, two empty
    q, off = _query_objects(db, obj, n_obj, [120, 0, 1, 200, 37, 0, 150, 3, 100], 3102)
    ref = oracle.object_scores(db, obj, n_obj, q, off)
    got = _gpu(qd, db, obj, n_obj, q, off)
    assert np.array_equal(got, ref)
    assert np.isinf(got[:, [4, 8]][[0, 2, 3, 4, 6, 7, 8]]).all()
    assert (got[[1, 5]] == 0).all()


def test_exact_copies_and_source_object(qd):
    sizes = [400] * 8
    db, obj = _objects(sizes, 3111)
    copies = db[obj == 5][:40]
    got = _gpu(qd, db, obj, 8, copies, np.array([0, 40], np.uint64))
    assert got[0, 5] == 0.0 and (np.delete(got[0], 5) > 0).all()
    q, off = _query_objects(db, obj, 8, [60] * 16, 3112)
    got = _gpu(qd, db, obj, 8, q, off)
    assert np.array_equal(got, oracle.object_scores(db, obj, 8, q, off))
    assert (got.argmin(1) == np.arange(16) % 8).all()


def test_edge_cases(qd):
    import torch
    db, obj = _objects([300, 20], 3121)
    q, off = _query_objects(db, obj, 2, [5, 7], 3122)
    # no query descriptors: every score is 0
    empty_q = np.zeros((0, 64), np.uint64)
    got = _gpu(qd, db, obj, 2, empty_q, np.zeros(4, np.uint64))
    assert got.shape == (3, 2) and (got == 0).all()
    # no database rows: +inf for every non-empty query object
    none = qd.object_scores(torch.zeros((0, 64), dtype=torch.int64, device="cuda:0"),
                            torch.zeros(0, dtype=torch.int16, device="cuda:0"), 3, _t(q), _t(off, np.int64))
    assert np.isinf(none.cpu().numpy()).all()
    # every row of an id >= n_obj: the same
    assert np.isinf(_gpu(qd, db, np.full(len(db), 9, np.uint16), 2, q, off)).all()
    # one object, one row, one descriptor
    one = db[:1]
    assert np.array_equal(_gpu(qd, one, np.zeros(1, np.uint16), 1, q[:1], np.array([0, 1], np.uint64)),
                          oracle.object_scores(one, np.zeros(1, np.uint16), 1, q[:1], np.array([0, 1], np.uint64)))
    # all-zero and all-one descriptors
    ext = np.concatenate([np.zeros((1, 64), np.uint64), np.full((1, 64), np.uint64(0xFFFFFFFFFFFFFFFF)), q])
    eoff = np.array([0, 1, 2, len(ext)], np.uint64)
    assert np.array_equal(_gpu(qd, db, obj, 2, ext, eoff), oracle.object_scores(db, obj, 2, ext, eoff))
    # invalid arguments
    with pytest.raises(qd.QDError):
        qd.object_scores(_t(db), _t(obj, np.int16), 0, _t(q), _t(off, np.int64))
    with pytest.raises(qd.QDError):
        qd.object_scores(_t(db), _t(obj, np.int16), 65537, _t(q), _t(off, np.int64))


def test_several_batches_many_objects(qd):
    # 65,536 objects: a batch holds 4,096 descriptors, so 9,000 descriptors take
    # three batches and query objects straddle the batch ends
    n_obj = 65536
    sizes = np.zeros(n_obj, np.int64)
    sizes[[0, 1, 17, 300, 4095, 65535]] = [500, 260, 1, 999, 256, 700]
    db, obj = _objects(sizes, 3131)
    q, _ = synth.gen_queries(db, 9000, 3132, 0.1, 0.6)
    off = np.array([0, 4000, 4095, 4097, 4097, 8191, 8192, 8193, 9000], np.uint64)
    ref = oracle.object_scores(db, obj, n_obj, q, off)
    got = _gpu(qd, db, obj, n_obj, q, off)
    assert np.array_equal(got, ref)


def test_retrieval_workload_sampled(qd):
    # the retrieval workload's database (300 objects x 5,000 rows); scores of
    # all 128 query objects on the GPU, two small ones checked by the oracle,
    # and the source object ranks first for every query object
    n_obj, per = 300, 5000
    db = synth.gen_db(n_obj * per, 1002)
    obj = (np.arange(n_obj * per) // per).astype(np.uint16)
    off, rows, qobj = synth.gen_query_objects(n_obj, per, 128, 1003, 200, 4000)
    q, _ = synth.gen_queries(db, len(rows), 1004, 0.2, 0.7, src=rows)
    got = _gpu(qd, db, obj, n_obj, q, off)
    assert (got.argmin(1) == qobj).all()
    sizes = np.diff(off)
    pick = np.sort(np.argsort(sizes, kind="stable")[:2])  # two of the smallest, in one oracle call
    sub = np.concatenate([q[int(off[g]):int(off[g + 1])] for g in pick])
    soff = np.concatenate([[0], np.cumsum(sizes[pick])]).astype(np.uint64)
    ref = oracle.object_scores(db, obj, n_obj, sub, soff)
    assert np.array_equal(got[pick], ref)


def _rows_gpu(qd, s, normalize=True):
    t = _t(np.ascontiguousarray(s, np.float64))
    best = qd.score_rows(t, normalize)
    return best.cpu().numpy(), t.cpu().numpy()


@pytest.mark.parametrize("n_obj", [1, 7, 300, 1000, 65536])
def test_score_rows_match_oracle(qd, n_obj):
    # integer-valued scores (many ties), +inf entries, a constant row, an all-inf row
    vals = synth.uniform_f32(9 * n_obj, 3141 + n_obj, 0.0, 20.0).astype(np.int64).astype(np.float64)
    s = vals.reshape(9, n_obj)
    s[1, ::3] = np.inf
    s[2] = 4.0
    s[3] = np.inf
    s[4, -1] = 0.5
    for normalize in (True, False):
        best, norm = _rows_gpu(qd, s, normalize)
        rbest, rnorm = oracle.score_rows(s, normalize)
        assert np.array_equal(best, rbest)
        assert np.array_equal(norm, rnorm)


def test_confusion_rows_of_computed_scores(qd):
    sizes = [700, 256, 257, 1, 0, 513, 90, 300, 0, 1024, 45, 600, 255, 380]
    db, obj = _objects(sizes, 3101, extra_none=77)
    q, off = _query_objects(db, obj, len(sizes), [120, 0, 1, 200, 37, 0, 150, 3, 100], 3102)
    s = qd.object_scores(_t(db), _t(obj, np.int16), len(sizes), _t(q), _t(off, np.int64))
    best = qd.score_rows(s)
    rbest, rnorm = oracle.score_rows(oracle.object_scores(db, obj, len(sizes), q, off))
    assert np.array_equal(best.cpu().numpy(), rbest)
    assert np.array_equal(s.cpu().numpy(), rnorm)


def test_score_rows_argument_errors(qd):
    import torch
    with pytest.raises(ValueError):
        qd.score_rows(torch.zeros((2, 3), dtype=torch.float32, device="cuda:0"))
    assert qd.score_rows(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0")).shape == (0,)
