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


def _hand_params():
    """A network worked out by hand: every weight is zero except a few, all
    exact in bfloat16.  Query bit b = 64*3 + 5 (image row 3, column 5) drives
    hidden unit 0 up (+2) and unit 1 down (-3, below its bias of +1, so its
    ReLU clips it); feature 4 adds 0.5 * f4 to unit 0.  In the second layer
    unit 0 feeds output unit 0 (x1.5, bias -3/16) and output unit 1 (x-1,
    clipped); a clipped unit 1 would add x10 to output unit 0.  The score is
    0.5 * h2[0] + 7 * h2[1] + 1/4."""
    W = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    b = 64 * 3 + 5
    W["W1q"][b, 0], W["W1q"][b, 1] = 2.0, -3.0
    W["b1"][1] = 1.0
    W["W1f"][4, 0] = 0.5
    W["W2"][0, 0], W["W2"][1, 0], W["W2"][0, 1] = 1.5, 10.0, -1.0
    W["b2"][0] = -0.1875
    W["w3"][0], W["w3"][1] = 0.5, 7.0
    W["b3"][0] = 0.25
    return mlp.pack(W).astype(np.float32), b


def test_forward_on_a_hand_worked_network():
    p, b = _hand_params()
    q = np.zeros((3, 64), np.uint64)
    q[0, 3] = np.uint64(1) << np.uint64(5)                              # bit b only
    q[1, 3] = np.uint64(1) << np.uint64(5)
    q[1, 40] = np.uint64(1) << np.uint64(63)                            # plus a bit with zero weights
    q[2, 5] = np.uint64(1) << np.uint64(3)                              # row 5, column 3: not bit b
    assert mlp.query_bits(q)[0].nonzero()[0].tolist() == [b]
    feat = np.zeros((3, mlp.NF), np.float32)
    feat[:, 4] = 0.25
    s, c = mlp.forward(p, q, [0, 1, 2], feat)
    # queries 0 and 1: z1 = [2 + 0.125, -3 + 1] -> h1 = [2.125, 0];
    # z2 = [1.5 * 2.125 - 0.1875, -2.125] -> h2 = [3, 0]; s = 0.5 * 3 + 0.25
    assert s[0] == 1.75 and s[1] == 1.75
    assert c["h1"][0, 0] == 2.125 and c["z1"][0, 1] == -2.0 and c["h1"][0, 1] == 0.0
    # query 2 lacks bit b: h1 = [0.125, 1]; z2[0] = 1.5 * 0.125 + 10 * 1 - 0.1875 = 10,
    # z2[1] = -0.125 -> 0; s = 0.5 * 10 + 0.25
    assert s[2] == 5.25


def test_gradient_on_a_hand_worked_network():
    p, b = _hand_params()
    q = np.zeros((1, 64), np.uint64)
    q[0, 3] = np.uint64(1) << np.uint64(5)
    feat = np.zeros((1, mlp.NF), np.float32)
    feat[0, 4] = 0.25
    loss, g = mlp.loss_and_grad(p, q, [0], feat, [1.0])
    ds = 1.0 / (1.0 + np.exp(-1.75)) - 1.0  # d loss / d s for label 1 at s = 1.75
    assert np.isclose(loss, np.log1p(np.exp(-1.75)), rtol=1e-14)
    G = mlp.unpack(g.astype(np.float64), round_bf16=False)
    # only the paths through the unclipped units 0 (layer 1) and 0 (layer 2) carry gradient
    assert np.isclose(G["b3"][0], ds, rtol=1e-14)
    assert np.isclose(G["w3"][0], 3.0 * ds, rtol=1e-14) and G["w3"][1] == 0.0
    assert np.isclose(G["b2"][0], 0.5 * ds, rtol=1e-14) and G["b2"][1] == 0.0
    assert np.isclose(G["W2"][0, 0], 0.5 * ds * 2.125, rtol=1e-14)
    assert G["W2"][1, 0] == 0.0 and G["W2"][0, 1] == 0.0
    assert np.isclose(G["b1"][0], 0.75 * ds, rtol=1e-14) and G["b1"][1] == 0.0
    assert np.isclose(G["W1q"][b, 0], 0.75 * ds, rtol=1e-14) and G["W1q"][b, 1] == 0.0
    assert np.count_nonzero(G["W1q"]) == 1                     # only the query's one set bit, unit 0
    assert np.isclose(G["W1f"][4, 0], 0.75 * ds * 0.25, rtol=1e-14)
    assert np.count_nonzero(G["W1f"]) == 1                     # the other features are zero
    assert sum(np.count_nonzero(v) for v in G.values()) == 7
