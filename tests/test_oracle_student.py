"""Pins of the student oracle (oracle/student.py) and of the oracle's
affine-last-layer model flag, against facts that do not come from the
oracle itself: published generator outputs, closed forms of Adam, finite
differences, exact least-squares recovery, sampling statistics, and a second
implementation of the student forward (the C oracle's generic layer code)."""
import json
import os

import numpy as np
import pytest

from paper_2005_00223_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def S():
    from oracle import student
    return student


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


def test_splitmix64_published_vectors(S):
    g = json.load(open(os.path.join(HERE, "golden", "splitmix64.json")))
    for v in g["vectors"]:
        out = S.splitmix64(v["seed"], np.arange(3))
        if "outputs_hex" in v:
            assert [int(x) for x in out] == [int(h, 16) for h in v["outputs_hex"]]
        else:
            assert [int(x) for x in out] == [int(d) for d in v["outputs_dec"]]


def test_round16_textbook_values(S):
    # 1/3 in binary16 is 0x3555, in bfloat16 0x3EAB; halfway cases go to even
    assert S.round16(1.0 / 3.0, 0) == 0.333251953125
    assert S.round16(1.0 / 3.0, 1) == 0.333984375
    assert S.round16(1.0 + 2.0 ** -11, 0) == 1.0
    assert S.round16(1.0 + 3 * 2.0 ** -11, 0) == 1.0 + 2.0 ** -9
    assert S.round16(1.0 + 2.0 ** -8, 1) == 1.0
    assert S.round16(1.0 + 3 * 2.0 ** -8, 1) == 1.0 + 2.0 ** -6


def _water():
    w = synth.workload("water192")
    return w, w["spec"]


def test_blob_v1_equals_v2_with_flag_off(O):
    w, spec = _water()
    b1 = synth.pack_blob(spec)
    import struct
    # the same model written as version 2 with emb_out_linear = 0
    head = b1[:8] + struct.pack("<q", 2) + b1[16:48] + struct.pack("<q", 0) + b1[48:]
    r1 = O.Oracle(b1).eval(w["coords"], w["types"], w["box"])
    r2 = O.Oracle(head).eval(w["coords"], w["types"], w["box"])
    assert r1["energy"] == r2["energy"]
    assert np.array_equal(r1["force"], r2["force"])


def test_affine_last_layer_is_linear_in_its_weights(O):
    """With the flag set, G(s) is linear in (W3, b3): a tanh there would
    break superposition."""
    w, spec = _water()
    P = synth.random_student_params(spec, 3).astype(np.float64)
    Q = synth.random_student_params(spec, 4).astype(np.float64)
    npar = synth.student_np(spec.M1)
    w3 = slice(npar - 33 * spec.M1, npar)
    PQ = P.copy()
    PQ[:, w3] = 0.7 * P[:, w3] - 1.9 * Q[:, w3]
    Pq = P.copy()
    Pq[:, w3] = Q[:, w3]
    oa, ob, oc = (O.Oracle(synth.pack_blob(synth.student_spec(spec, X))) for X in (P, Pq, PQ))
    for s in (0.0, 0.05, 0.17, 0.33):
        for t in range(2):
            for u in range(2):
                ga, gb, gc = oa.embed(t, u, s), ob.embed(t, u, s), oc.embed(t, u, s)
                np.testing.assert_allclose(gc, 0.7 * ga - 1.9 * gb, rtol=1e-12, atol=1e-12)


def test_student_forward_matches_c_oracle(S, O):
    """oracle.student.forward (numpy, student-specific) against the C
    oracle's generic skip-rule layer code on the same student blob."""
    w, spec = _water()
    P = synth.random_student_params(spec, 5)
    o = O.Oracle(synth.pack_blob(synth.student_spec(spec, P)))
    s = np.linspace(0.0, 0.45, 23)
    for net in range(4):
        G, _ = S.forward(P[net].astype(np.float64), s, spec.M1)
        ref = np.array([o.embed(net // 2, net % 2, x) for x in s])
        np.testing.assert_allclose(G, ref, rtol=1e-13, atol=1e-13)


def test_student_model_forces_are_minus_gradient(O):
    """Central differences of the oracle energy of a student model
    (affine last layer) against its analytic forces."""
    w, spec = _water()
    P = synth.random_student_params(spec, 6)
    o = O.Oracle(synth.pack_blob(synth.student_spec(spec, P)))
    x = w["coords"].copy()
    r = o.eval(x, w["types"], w["box"])
    rng = np.random.default_rng(0)
    h = 1e-5
    worst = 0.0
    for k in rng.choice(len(x), 6, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, a] += h
            xm[k, a] -= h
            fd = -(o.eval(xp, w["types"], w["box"])["energy"] - o.eval(xm, w["types"], w["box"])["energy"]) / (2 * h)
            worst = max(worst, abs(fd - r["force"][k, a]))
    scale = np.abs(r["force"]).max()
    assert worst < 1e-6 * max(scale, 1.0)


def test_loss_gradient_matches_central_differences(S):
    rng = np.random.default_rng(1)
    M1 = 100
    p = rng.normal(size=S.layout(M1)["np"]) * 0.3
    s = rng.uniform(0, 0.4, size=24)
    wts = (rng.uniform(size=24) > 0.2).astype(float)
    Gt = rng.normal(size=(24, M1))
    L0, g = S.loss_grad(p, s, wts, Gt, M1)
    h = 1e-6
    idx = rng.choice(len(p), 80, replace=False)
    idx = np.concatenate([idx, [0, 16, 32, 544, 576, len(p) - 1]])
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (S.loss_grad(pp, s, wts, Gt, M1)[0] - S.loss_grad(pm, s, wts, Gt, M1)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])
    # the loss itself, by its definition
    G, _ = S.forward(p, s, M1)
    assert np.isclose(L0, (wts[:, None] * (G - Gt) ** 2).sum() / (M1 * wts.sum()), rtol=1e-14)


def test_adam_closed_forms(S):
    rng = np.random.default_rng(2)
    g = rng.normal(size=50)
    p0 = rng.normal(size=50)
    lr, eps = 1e-3, 1e-8
    # the bias-corrected first step moves every parameter by lr g/(|g|+eps)
    p1, m, v = S.adam(p0, g, np.zeros(50), np.zeros(50), 1, lr=lr, eps=eps)
    np.testing.assert_allclose(p0 - p1, lr * g / (np.abs(g) + eps), rtol=1e-12)
    # under a constant gradient the corrected moments are g and g^2 at every step
    p = p0.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 8):
        q, m, v = S.adam(p, g, m, v, t, lr=lr, eps=eps)
        np.testing.assert_allclose(p - q, lr * g / (np.abs(g) + eps), rtol=1e-9)
        p = q


def test_refit_recovers_an_exact_affine_target(S):
    rng = np.random.default_rng(3)
    M1 = 100
    p = rng.normal(size=S.layout(M1)["np"])
    p[:16] *= 5.0
    s = rng.uniform(0, 0.4, size=3000)
    wts = np.ones(3000)
    Xs = rng.normal(size=(32, M1)) * 0.3
    bs = rng.normal(size=M1)
    _, (_, _, h2) = S.forward(p, s, M1)
    Gt = h2 @ Xs + bs
    q = S.refit(p, s, wts, Gt, M1)
    W1, b1, W2, b2, W3, b3 = S.unpack(q, M1)
    G, _ = S.forward(q, s, M1)
    assert np.abs(G - Gt).max() < 1e-9
    # rounded variant: W3 holds FP16 values and the residual has zero mean
    q16 = S.refit(p, s, wts, Gt, M1, quant=0)
    W3q = S.unpack(q16, M1)[4]
    assert np.array_equal(W3q, S.round16(W3q, 0))
    G16, _ = S.forward(q16, s, M1)
    assert np.abs((Gt - G16).mean(axis=0)).max() < 1e-12


def test_sampler_is_uniform_over_real_pairs(S, O):
    """Hits per centre atom follow its real-neighbour count (chi-square),
    samples do not depend on how they are batched, and every drawn s is the
    s of a real neighbour slot."""
    w = synth.workload("cu_cells5")
    spec = w["spec"]
    o = O.Oracle(synth.pack_blob(spec))
    r = o.eval(w["coords"], w["types"], w["box"], intermediates=True)
    sel = np.array(spec.sel)
    n = 200000
    s, wt, ci, sl = S.sample(w["types"], r["nreal"], r["rt"], sel, 1, 7, 0, 0, n)
    assert wt.all()
    assert np.all(sl < r["nreal"][ci, 0])
    assert np.array_equal(s, r["rt"][ci, sl, 0])
    hits = np.bincount(ci, minlength=len(w["types"]))
    expect = n * r["nreal"][:, 0] / r["nreal"][:, 0].sum()
    chi2 = ((hits - expect) ** 2 / expect).sum()
    dof = len(hits) - 1
    assert abs(chi2 - dof) < 5 * np.sqrt(2 * dof), (chi2, dof)
    s2 = S.sample(w["types"], r["nreal"], r["rt"], sel, 1, 7, 0, 1000, 500)[0]
    assert np.array_equal(s2, s[1000:1500])


def test_sampler_without_pairs_gives_zero_weight(S):
    types = np.array([0, 0, 0])
    nreal = np.zeros((3, 2), dtype=np.int32)
    rt = np.zeros((3, 4, 4))
    s, wt, _, _ = S.sample(types, nreal, rt, np.array([2, 2]), 2, 1, 1, 0, 64)
    assert not wt.any() and not s.any()
    # no centre of type 1 at all
    s, wt, _, _ = S.sample(types, nreal, rt, np.array([2, 2]), 2, 1, 2, 0, 64)
    assert not wt.any()


def test_round_spec16_rounds_only_the_16bit_weights():
    """The rounded-weight model used to separate weight rounding from kernel
    arithmetic: embedding layers after the first and the first two fitting
    layers are rounded (idempotently, to representable 16-bit values); the
    first embedding layer, later fitting layers and all biases are not."""
    from oracle import student as S
    spec = synth.water_model(0)
    for quant, dt in ((0, np.float16), (1, None)):
        q = S.round_spec16(spec, quant)
        for t in range(spec.ntypes):
            for u in range(spec.ntypes):
                assert np.array_equal(q.emb_W[t][u][0], spec.emb_W[t][u][0])
                for l in range(1, len(spec.emb)):
                    W = q.emb_W[t][u][l]
                    assert not np.array_equal(W, spec.emb_W[t][u][l])
                    assert np.array_equal(S.round16(W, quant), W)
                    if dt is not None:
                        assert np.array_equal(W.astype(dt).astype(np.float64), W)
                    else:  # bfloat16: the low 16 bits of the float32 pattern are zero
                        assert np.all((W.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
                    assert np.abs(W - spec.emb_W[t][u][l]).max() <= 2.0 ** (-8 if quant else -11) * np.abs(
                        spec.emb_W[t][u][l]).max()
                for l in range(len(spec.emb)):
                    assert np.array_equal(q.emb_b[t][u][l], spec.emb_b[t][u][l])
            for l in range(len(spec.fit_W[t])):
                same = np.array_equal(q.fit_W[t][l], spec.fit_W[t][l])
                assert same == (l >= 2)
