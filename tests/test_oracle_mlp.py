"""Pins for the MLP oracle: finite differences, closed-form special cases,
and the feature definitions on hand-made nodes."""
import numpy as np

import synth
from oracle import mlp


def _params(seed, scale=0.05):
    return synth.uniform_f32(mlp.NPARAMS, seed, -scale, scale)


def _batch(seed, nq=3, per=4):
    q = synth.gen_db(nq, seed)
    pair_q = np.repeat(np.arange(nq), per)
    rng = np.random.default_rng(seed)
    feat = rng.random((nq * per, mlp.NF)).astype(np.float32)
    y = (rng.random(nq * per) < 0.4).astype(np.float64)
    return q, pair_q, feat, y


def test_gradient_matches_finite_differences():
    p = _params(1, 0.1).astype(np.float64)
    q, pair_q, feat, y = _batch(2)
    loss, g = mlp.loss_and_grad(p, q, pair_q, feat, y, round_bf16=False)
    rng = np.random.default_rng(3)
    qbits = np.flatnonzero(mlp.query_bits(q).any(0))
    # probe parameters in every block, W1q rows only where some query bit is set
    o = 0
    probes = []
    for name, shape in mlp.SIZES:
        n = int(np.prod(shape))
        if name == "W1q":
            rows = rng.choice(qbits, 6)
            cols = rng.integers(0, mlp.H, 6)
            probes += list(o + rows * mlp.H + cols)
        else:
            probes += list(o + rng.integers(0, n, min(n, 6)))
        o += n
    eps = 1e-6
    for i in probes:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        lp, _ = mlp.loss_and_grad(pp, q, pair_q, feat, y, round_bf16=False)
        lm, _ = mlp.loss_and_grad(pm, q, pair_q, feat, y, round_bf16=False)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_zero_weights_give_the_bias_and_its_gradient():
    p = np.zeros(mlp.NPARAMS, np.float32)
    p[-1] = 0.75  # b3
    q, pair_q, feat, y = _batch(4)
    s, _ = mlp.forward(p, q, pair_q, feat)
    assert np.allclose(s, 0.75)
    loss, g = mlp.loss_and_grad(p, q, pair_q, feat, y)
    sig = 1 / (1 + np.exp(-0.75))
    assert np.isclose(g[-1], np.mean(sig - y))
    assert np.isclose(loss, np.mean(np.log1p(np.exp(0.75)) - y * 0.75))
    assert np.count_nonzero(g[:-1]) == 0  # ReLU of zero blocks every other path


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.1415926], np.float32)
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0          # halfway rounds to the even mantissa
    assert r[2] == 1.0 + 2 ** -6                 # halfway rounds up to even
    assert r[3] == -2.5 and abs(r[4] - 3.140625) < 1e-12


def test_features_on_hand_made_nodes():
    # query: row 0 bits 0-9 and row 63 bits 0-9 (20 bits); node OR covers row 0 only
    q = synth.from_bits(1, [list(range(10)) + [64 * 63 + i for i in range(10)]])
    orimg = synth.from_bits(3, [list(range(64)), list(range(64)), [64 * 63 + 5]])
    child = np.array([[1, 2], [-1, -1], [-1, -1]])
    parent = np.array([-1, 0, 0])
    depth = np.array([0, 1, 1])
    count = np.array([64, 32, 32])
    f = mlp.features(q, orimg, child, parent, depth, count, [0, 0], [1, 2])
    # node 1: covers the 10 row-0 bits, misses the 10 row-63 bits
    assert np.isclose(f[0, 0], 0.5) and np.isclose(f[0, 1], 0.5)
    assert np.isclose(f[0, 2], 64 / 4096) and np.isclose(f[0, 3], 19 / 20)  # sibling covers 1 bit
    assert f[0, 6] == 1.0 and f[0, 7] == 1.0 and np.isclose(f[0, 5], 5 / 24)
    assert np.isclose(f[0, 9], 54 / 4096)
    assert np.isclose(f[0, 10 + 0], 0.0) and np.isclose(f[0, 21 + 0], 0.5)    # band of rows 0-5
    assert np.isclose(f[0, 10 + 10], 0.5) and np.isclose(f[0, 21 + 10], 0.0)  # band of rows 60-63
    # node 2: the dissimilar child covers one query bit
    assert np.isclose(f[1, 0], 19 / 20) and f[1, 7] == 0.0 and np.isclose(f[1, 3], 0.5)
