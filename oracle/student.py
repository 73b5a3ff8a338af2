"""FP64 reference of the student embedding net -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never does, and it imports nothing from the HIP
package.  Plain numpy, float64, no blocking or fusion, so that each step can
be read against its definition.

The student (not part of the paper) stands in for the embedding nets of
Fig. 1(e,f): per (centre type, neighbour type) pair a smaller net
1 -> 16 (tanh) -> 32 (tanh, doubling skip) -> M1 (affine), fitted to the
full net's own G(s) at neighbour distances of one configuration.

  sample()      which neighbour pairs are drawn: SplitMix64 (Steele, Lea and
                Flood, "Fast splittable pseudorandom number generators",
                OOPSLA 2014) as a counter-based generator, rejection sampling
                over (centre of type t, slot below sel_u)
  forward()     the student net
  loss_grad()   mean squared error over samples and outputs, and its
                gradient by the chain rule
  adam()        one Adam update (Kingma and Ba, ICLR 2015, Algorithm 1)
  refit()       least squares of the affine output layer on the hidden
                features (h2, 1), optionally with the 16-bit rounding of W2
                and W3 that the mixed-precision kernels apply
"""
from __future__ import annotations

import numpy as np

SH1, SH2 = 16, 32
ATTEMPTS = 32
GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def layout(M1: int) -> dict:
    """Offsets of the packed parameters W1[16] b1[16] W2[16][32] b2[32]
    W3[32][M1] b3[M1] (row = input feature)."""
    o = {"w1": 0, "b1": SH1, "w2": 2 * SH1}
    o["b2"] = o["w2"] + SH1 * SH2
    o["w3"] = o["b2"] + SH2
    o["b3"] = o["w3"] + SH2 * M1
    o["np"] = o["b3"] + M1
    return o


def unpack(p, M1):
    o = layout(M1)
    p = np.asarray(p, dtype=np.float64)
    return (p[o["w1"]:o["b1"]], p[o["b1"]:o["w2"]], p[o["w2"]:o["b2"]].reshape(SH1, SH2),
            p[o["b2"]:o["w3"]], p[o["w3"]:o["b3"]].reshape(SH2, M1), p[o["b3"]:o["np"]])


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(W3), np.ravel(b3)])


# ---------------------------------------------------------------------------
# SplitMix64: output number ctr (0-based) of the stream seeded with seed is
# mix(seed + (ctr+1) * gamma) with the published finaliser
# ---------------------------------------------------------------------------
def splitmix64(seed, ctr):
    """Vectorised over ctr (numpy uint64, arithmetic modulo 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(ctr, dtype=np.uint64) + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sample(types, nreal, rt, sel, ntypes, seed, net, q0, batch):
    """Samples q0 .. q0+batch-1 of net (t, u) = divmod(net, ntypes).

    types [N]; nreal [N][ntypes] real neighbours per type; rt [N][sum sel][4]
    environment rows (rt[..., 0] = s).  Attempt a of sample q takes
    x = splitmix64(seed, ((net << 40) + q) * 32 + a), centre = the
    ((x >> 32) * count_t >> 32)-th atom of type t in index order,
    slot = (x & 0xffffffff) * sel_u >> 32, and keeps it when slot is below
    that centre's real count; no success in 32 attempts gives weight 0.
    Returns (s [batch], weight [batch], centre [batch], slot [batch])."""
    t, u = divmod(int(net), int(ntypes))
    centres_t = np.nonzero(np.asarray(types) == t)[0]
    count, selu = len(centres_t), int(sel[u])
    off_u = int(np.sum(sel[:u]))
    s = np.zeros(batch)
    w = np.zeros(batch)
    ci = np.full(batch, -1, dtype=np.int64)
    sl = np.full(batch, -1, dtype=np.int64)
    if count == 0 or selu == 0:
        return s, w, ci, sl
    q = np.arange(q0, q0 + batch, dtype=np.uint64)
    a = np.arange(ATTEMPTS, dtype=np.uint64)
    ctr = ((np.uint64(net) << np.uint64(40)) + q[:, None]) * np.uint64(ATTEMPTS) + a[None, :]
    x = splitmix64(seed, ctr)
    k = ((x >> np.uint64(32)) * np.uint64(count)) >> np.uint64(32)
    slot = ((x & np.uint64(0xFFFFFFFF)) * np.uint64(selu)) >> np.uint64(32)
    atom = centres_t[k.astype(np.int64)]
    ok = slot.astype(np.int64) < np.asarray(nreal)[atom, u]
    has = ok.any(axis=1)
    first = np.argmax(ok, axis=1)
    rows = np.nonzero(has)[0]
    ci[rows] = atom[rows, first[rows]]
    sl[rows] = slot[rows, first[rows]].astype(np.int64)
    s[rows] = np.asarray(rt)[ci[rows], off_u + sl[rows], 0]
    w[rows] = 1.0
    return s, w, ci, sl


# ---------------------------------------------------------------------------
# the student net and its squared error
# ---------------------------------------------------------------------------
def forward(p, s, M1):
    """G(s) [B, M1] and the hidden activations (t1, t2, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, M1)
    s = np.asarray(s, dtype=np.float64)
    t1 = np.tanh(s[:, None] * W1[None, :] + b1[None, :])        # 1 -> 16, no skip
    t2 = np.tanh(t1 @ W2 + b2)                                   # 16 -> 32
    h2 = np.concatenate([t1, t1], axis=1) + t2                   # doubling skip
    G = h2 @ W3 + b3                                             # affine output
    return G, (t1, t2, h2)


def loss_grad(p, s, w, Gt, M1):
    """L = sum_q w_q sum_o (G_s(s_q)_o - Gt_qo)^2 / (M1 sum_q w_q) and dL/dp."""
    W1, b1, W2, b2, W3, b3 = unpack(p, M1)
    w = np.asarray(w, dtype=np.float64)
    G, (t1, t2, h2) = forward(p, s, M1)
    denom = M1 * max(w.sum(), 1.0)
    r = w[:, None] * (G - Gt)
    L = float((r * r).sum() / denom)
    dG = 2.0 * r / denom
    dW3 = h2.T @ dG
    db3 = dG.sum(axis=0)
    dh2 = dG @ W3.T
    dz2 = dh2 * (1.0 - t2 * t2)
    dW2 = t1.T @ dz2
    db2 = dz2.sum(axis=0)
    dt1 = dz2 @ W2.T + dh2[:, :SH1] + dh2[:, SH1:]
    dz1 = dt1 * (1.0 - t1 * t1)
    dW1 = (np.asarray(s)[:, None] * dz1).sum(axis=0)
    db1 = dz1.sum(axis=0)
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Update number t (1-based): returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# output-layer least squares
# ---------------------------------------------------------------------------
def round16(x, quant):
    """Round to nearest even in FP16 (quant 0) or BF16 (quant 1) through
    float32; quant < 0 returns x."""
    x32 = np.asarray(x, dtype=np.float32)
    if quant == 0:
        return x32.astype(np.float16).astype(np.float64)
    if quant == 1:
        u = x32.view(np.uint32).astype(np.uint64)
        u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


def round_spec16(spec, quant, n_fit16=2):
    """A copy of the model spec with the weights a 16-bit policy holds in
    16 bits rounded (quant 0 FP16, 1 BF16), kept in FP64: the embedding
    layers after the first (the first is a rank-1 layer kept in FP32) and
    the first n_fit16 fitting layers.  Evaluating it with the FP64 oracle
    separates the effect of the weight rounding from the arithmetic of the
    16-bit kernels."""
    import copy
    q = copy.deepcopy(spec)
    for t in range(spec.ntypes):
        for u in range(spec.ntypes):
            for l in range(1, len(spec.emb)):
                q.emb_W[t][u][l] = round16(spec.emb_W[t][u][l], quant)
        for l in range(n_fit16):
            q.fit_W[t][l] = round16(spec.fit_W[t][l], quant)
    return q


def refit(p, s, w, Gt, M1, quant=-1):
    """Least squares of [h2(s), 1] X = Gt over the weighted samples
    (numpy lstsq); with quant >= 0, W2 is rounded before the features are
    formed, W3 after the solve, and b3 is the mean residual given W3.
    Returns the packed parameters with W2, W3, b3 replaced."""
    W1, b1, W2, b2, W3, b3 = unpack(p, M1)
    W2 = round16(W2, quant)
    q = pack(W1, b1, W2, b2, W3, b3)
    _, (_, _, h2) = forward(q, s, M1)
    keep = np.asarray(w) > 0
    A = np.concatenate([h2[keep], np.ones((keep.sum(), 1))], axis=1)
    X = np.linalg.lstsq(A, Gt[keep], rcond=None)[0]
    W3n = round16(X[:SH2], quant)
    b3n = (Gt[keep] - h2[keep] @ W3n).mean(axis=0)
    return pack(W1, b1, W2, b2, W3n, b3n)
