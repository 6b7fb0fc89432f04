"""CPU oracle for the frontier-order MLP (TEST INFRASTRUCTURE ONLY).

Plain numpy in float64: node features, forward pass, binary cross-entropy
and its gradient, written from their definitions.  The GPU library computes
the same network with BF16 weights and FP32 accumulation; this oracle uses
the same BF16-rounded weights and inputs and exact float64 arithmetic
otherwise.  Shares no code with the GPU library.

Network: x = [query bits (4096); features f (32)];
h1 = ReLU(x W1 + b1); h2 = ReLU(h1 W2 + b2); s = h2 . w3 + b3.
Parameter vector layout (float32, 1,123,073 values), matrices [input][output]:
W1q 4096x256, W1f 32x256, b1 256, W2 256x256, b2 256, w3 256, b3 1.
"""
import numpy as np

NB, NF, H = 4096, 32, 256
SIZES = [("W1q", (NB, H)), ("W1f", (NF, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)),
         ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even); returns float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def unpack(params, round_bf16=True):
    assert np.shape(params) == (NPARAMS,)
    if round_bf16:
        p = bf16_round(np.asarray(params, dtype=np.float32))
    else:
        p = np.asarray(params, dtype=np.float64)  # exact float64 (finite-difference checks)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def query_bits(q):
    """(nq, 64) uint64 -> (nq, 4096) float64 of 0/1, bit b = 64*row + col."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    return np.unpackbits(q.view(np.uint8), axis=1, bitorder="little").astype(np.float64)


def _popcount(a):
    return np.unpackbits(np.ascontiguousarray(a).view(np.uint8), axis=-1).sum(-1).astype(np.float64)


BANDS = [(6 * b, min(6 * b + 6, 64)) for b in range(11)]  # image rows of each band


def features(q, or_img, child, parent, depth, count, pair_q, pair_node):
    """32 features of each (query, node) pair, from their definitions."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.zeros((len(pair_q), NF))
    for p, (qi, nd) in enumerate(zip(pair_q, pair_node)):
        qq, oo = q[qi], or_img[nd]
        pq = max(_popcount(qq), 1.0)
        par = parent[nd]
        if par >= 0:
            sib = child[par][1] if child[par][0] == nd else child[par][0]
        else:
            sib = -1
        a_rows = np.array([_popcount(qq[r:r + 1] & ~oo[r:r + 1]) for r in range(64)])
        o_rows = np.array([_popcount(qq[r:r + 1] & oo[r:r + 1]) for r in range(64)])
        f = out[p]
        f[0] = a_rows.sum() / pq
        f[1] = o_rows.sum() / pq
        f[2] = _popcount(oo) / 4096.0
        f[3] = _popcount(qq & ~or_img[sib]) / pq if sib >= 0 else 0.0
        f[4] = depth[nd] / 32.0
        f[5] = np.log2(count[nd]) / 24.0
        f[6] = 1.0 if child[nd][0] < 0 else 0.0
        f[7] = 1.0 if (par >= 0 and child[par][0] == nd) else 0.0
        f[8] = _popcount(qq) / 512.0
        f[9] = _popcount(oo & ~qq) / 4096.0
        for b, (r0, r1) in enumerate(BANDS):
            f[10 + b] = a_rows[r0:r1].sum() / pq
            f[21 + b] = o_rows[r0:r1].sum() / pq
    return out


def forward(params, q, pair_q, feat, round_bf16=True):
    """Scores (logits) and the intermediate values of a batch of pairs."""
    W = unpack(params, round_bf16)
    qb = query_bits(q)[np.asarray(pair_q)]
    f = np.asarray(feat, dtype=np.float64)  # features are float32 inputs; used as given
    z1 = qb @ W["W1q"] + f @ W["W1f"] + W["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W["W2"] + W["b2"]
    h2 = np.maximum(z2, 0.0)
    s = h2 @ W["w3"] + W["b3"][0]
    return s, dict(qb=qb, f=f, z1=z1, h1=h1, z2=z2, h2=h2, W=W)


def loss_and_grad(params, q, pair_q, feat, y, round_bf16=True):
    """Mean binary cross-entropy of the logits against labels y, and its
    gradient with respect to every parameter (float64, parameter layout)."""
    s, c = forward(params, q, pair_q, feat, round_bf16)
    y = np.asarray(y, dtype=np.float64)
    n = len(s)
    loss = np.mean(np.logaddexp(0.0, s) - y * s)
    ds = (1.0 / (1.0 + np.exp(-s)) - y) / n
    W = c["W"]
    g = {}
    g["b3"] = np.array([ds.sum()])
    g["w3"] = c["h2"].T @ ds
    dz2 = np.outer(ds, W["w3"]) * (c["z2"] > 0)
    g["b2"] = dz2.sum(0)
    g["W2"] = c["h1"].T @ dz2
    dz1 = (dz2 @ W["W2"].T) * (c["z1"] > 0)
    g["b1"] = dz1.sum(0)
    g["W1f"] = c["f"].T @ dz1
    g["W1q"] = c["qb"].T @ dz1
    return loss, pack(g)
