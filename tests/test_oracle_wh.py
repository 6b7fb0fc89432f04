"""Pins for the oracle's Weighted Hamming distance (Eq. 1, Section 2.3).

The oracle is checked against hand-worked values, closed forms, the plain
Hamming distance and its identities, each computed here independently of the
oracle (numpy bit unpacking, exact fractions).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "wh_hand.txt")
NB = 4096


def _bits(spec):
    if spec == "-":
        return []
    if spec == "all":
        return list(range(NB))
    out = []
    for part in spec.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def _frac(expr):
    return sum((Fraction(t.strip()) for t in expr.split("+")), Fraction(0))


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, qs, ts, a, b, p, d = [x.strip() for x in line.split("|")]
        rows.append((name, _bits(qs), _bits(ts), int(a), int(b), int(p), _frac(d)))
    return rows


def _pop(x):
    return int(np.unpackbits(np.ascontiguousarray(x).view(np.uint8)).sum())


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[0])
def test_hand_worked_cases(case):
    name, qb, tb, A, B, P, d = case
    q, t = synth.from_bits(2, [qb, tb])
    assert oracle.wh_literal(q, t) == (A, B, P)
    # Eq. 1 in double agrees with the exact fraction
    assert abs(oracle.wh_eq1(A, B, P) - float(d)) <= 4e-16 * max(1.0, float(d))
    # the integer key is d * wA * wB exactly
    wa, wb = max(P, 1), max(NB - P, 1)
    assert Fraction(oracle.wh_key(A, B, P), wa * wb) == d
    # the reported float is the exact value rounded to float32 (within 1 ulp)
    assert abs(float(oracle.wh_dist(A, B, P)) - float(d)) <= float(np.spacing(np.float32(float(d))))


def _rand_descs(n, seed):
    return synth.gen_db(n, seed)


def test_identity_and_complement():
    db = _rand_descs(50, 11)
    for x in db:
        A, B, P = oracle.wh_literal(x, x)
        assert (A, B) == (0, 0) and oracle.wh_eq1(A, B, P) == 0.0
        nx = ~x
        A, B, P = oracle.wh_literal(x, nx)
        assert 0 < P < NB
        assert oracle.wh_eq1(A, B, P) == 2.0  # every bit is an error: P/P + (4096-P)/(4096-P)
        zero = np.zeros(64, np.uint64)
        A, B, P = oracle.wh_literal(x, zero)
        assert oracle.wh_eq1(A, B, P) == 1.0  # all query bits missed
        A, B, P = oracle.wh_literal(zero, x)
        assert P == 0 and Fraction(oracle.wh_key(A, B, P), 1 * NB) == Fraction(_pop(x), NB)


def test_superset_and_subset_closed_forms():
    rng = np.random.default_rng(5)
    db = _rand_descs(40, 12)
    for x in db:
        P = _pop(x)
        # extra bits e disjoint from q: d = |e| / (4096 - |q|)
        extra = np.zeros(64, np.uint64)
        free = [b for b in range(NB) if not (int(x[b >> 6]) >> (b & 63)) & 1]
        for b in rng.choice(free, size=17, replace=False):
            extra[b >> 6] |= np.uint64(1) << np.uint64(b & 63)
        A, B, Pq = oracle.wh_literal(x, x | extra)
        assert (A, B, Pq) == (0, 17, P)
        assert Fraction(oracle.wh_key(A, B, Pq), P * (NB - P)) == Fraction(17, NB - P)
        # missed bits m inside q: d = |m| / |q|
        setb = [b for b in range(NB) if (int(x[b >> 6]) >> (b & 63)) & 1]
        miss = np.zeros(64, np.uint64)
        for b in rng.choice(setb, size=9, replace=False):
            miss[b >> 6] |= np.uint64(1) << np.uint64(b & 63)
        A, B, Pq = oracle.wh_literal(x, x & ~miss)
        assert (A, B) == (9, 0)
        assert Fraction(oracle.wh_key(A, B, Pq), P * (NB - P)) == Fraction(9, P)


def test_hamming_identities_and_asymmetry():
    db = _rand_descs(60, 13)
    asym = 0
    for i in range(0, 60, 2):
        q, t = db[i], db[i + 1]
        A, B, P = oracle.wh_literal(q, t)
        assert A + B == _pop(q ^ t)            # plain Hamming distance
        assert A + _pop(q & t) == P == _pop(q)  # A + C = |q|
        assert B + _pop(q & t) == _pop(t)       # B + C = |t|
        A2, B2, P2 = oracle.wh_literal(t, q)
        assert (A2, B2) == (B, A)               # swapping roles swaps error types
        if oracle.wh_eq1(A, B, P) != oracle.wh_eq1(A2, B2, P2):
            asym += 1
    assert asym > 0  # Weighted Hamming is asymmetric in general


def test_bruteforce_counts_match_literal_loop(small_db, small_queries):
    q, _ = small_queries
    r = oracle.knn_brute(small_db[:500], q[:8], 20)
    for j in range(8):
        for s in range(20):
            A, B, P = oracle.wh_literal(q[j], small_db[r.idx[j, s]])
            assert (r.missed[j, s], r.extra[j, s]) == (A, B)
            assert r.dist[j, s] == np.float32(oracle.wh_dist(A, B, P))
