"""The no-allocation sequential search, through the C ABI, against the
sequential search that allocates its scratch (qd_knn_bruteforce) and the
oracle: bit-exact idx, missed, extra and dist on two calls in a row, the
second smaller than the first (the fixed scratch keeps the first call's
contents, which must not leak into the second)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda:0")


def _np(res):
    return [x.cpu().numpy() for x in res]


def _call(qd, db, q, k, out):
    import torch
    f = qd.lib().qd_knn_bruteforce_noalloc
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = f(p(db), db.shape[0], p(q), q.shape[0], k, *(p(t) for t in out), s)
    assert rc == 0, qd.lib().qd_last_error()
    return out


def test_noalloc_matches_allocating_search_on_two_calls():
    import torch
    import paper_2107_03368_amd as qd
    db = synth.gen_db(100_003, 1201)
    q, _ = synth.gen_queries(db, 700, 2201, 0.1, 0.6)
    dbt, qt = _t(db), _t(q)
    # outputs allocated once, as a caller that cannot allocate would hold them
    out = (torch.empty(700 * 64, dtype=torch.int32, device="cuda:0"),
           torch.empty(700 * 64, dtype=torch.int32, device="cuda:0"),
           torch.empty(700 * 64, dtype=torch.int32, device="cuda:0"),
           torch.empty(700 * 64, dtype=torch.float32, device="cuda:0"))
    cases = ((dbt, qt, 700, 50), (dbt[:9_999], qt[:37], 37, 10))  # the second call is smaller
    for n_db, n_q, nq, k in cases:
        got = _np(x[:nq * k].view(nq, k) for x in _call(qd, n_db, n_q, k, out))
        ref = _np(qd.knn_bruteforce(n_db, n_q, k))
        for a, b, what in zip(got, ref, ("idx", "missed", "extra", "dist")):
            assert np.array_equal(a, b), what
        rows = np.array([0, nq // 2, nq - 1])
        o = oracle.knn_brute(db[:n_db.shape[0]], q[rows], k)
        assert np.array_equal(got[0][rows].view(np.uint32), o.idx)
        assert np.array_equal(got[1][rows], o.missed)
        assert np.array_equal(got[2][rows], o.extra)
        assert np.array_equal(got[3][rows], o.dist)
    # the binding's wrapper gives the same results
    res = _np(qd.knn_bruteforce_noalloc(dbt[:9_999], qt[:37], 10))
    ref = _np(qd.knn_bruteforce(dbt[:9_999], qt[:37], 10))
    for a, b in zip(res, ref):
        assert np.array_equal(a, b)


def test_noalloc_rejects_lists_beyond_its_scratch():
    import paper_2107_03368_amd as qd
    db = _t(synth.gen_db(1000, 1202))
    q = _t(np.zeros((65_537, 64), np.uint64))
    with pytest.raises(qd.QDError) as e:
        qd.knn_bruteforce_noalloc(db, q, 64)
    assert e.value.code == -1 and "scratch" in str(e.value)
