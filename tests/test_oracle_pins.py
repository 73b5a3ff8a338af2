"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics, not against the oracle itself: brute force, closed forms,
finite differences, invariances and special cases.  CPU only."""
import json
import os

import numpy as np
import pytest

from paper_2005_00223_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def water(oracle_mod):
    w = synth.workload("water192")
    return w, oracle_mod.Oracle(synth.pack_blob(w["spec"]))


@pytest.fixture(scope="module")
def cu(oracle_mod):
    w = synth.workload("cu_cells5")
    return w, oracle_mod.Oracle(synth.pack_blob(w["spec"]))


# ---------------------------------------------------------------------------
# neighbour list (Section V-B: type, then distance; nearest sel kept; -1 pad;
# ties by index as in the packed key)
# ---------------------------------------------------------------------------
def _numpy_bruteforce_nlist(x, types, box, rc, sel):
    """Independent O(N^2) list straight from the definition."""
    x = x - box * np.floor(x / box)
    x[x >= box] = 0.0
    n = len(types)
    off = np.concatenate([[0], np.cumsum(sel)])
    nl = -np.ones((n, off[-1]), dtype=np.int32)
    nr = np.zeros((n, len(sel)), dtype=np.int32)
    for i in range(n):
        d = x - x[i]
        d = np.where(d > 0.5 * box, d - box, np.where(d < -0.5 * box, d + box, d))
        r = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
        idx = np.nonzero((r <= rc) & (np.arange(n) != i))[0]
        q = np.floor(r[idx] * 1e8).astype(np.uint64)
        order = np.lexsort((idx, q, types[idx]))
        idx, t = idx[order], types[idx][order]
        for u in range(len(sel)):
            ju = idx[t == u][: sel[u]]
            nl[i, off[u]:off[u] + ju.size] = ju
            nr[i, u] = ju.size
    return nl, nr


def test_nlist_numpy_bruteforce_water(water):
    w, o = water
    nl, nr, ovf = o.nlist(w["coords"], w["types"], w["box"])
    spec = w["spec"]
    nl2, nr2 = _numpy_bruteforce_nlist(w["coords"].copy(), w["types"], w["box"], spec.rcut, spec.sel)
    assert ovf == 0
    np.testing.assert_array_equal(nl, nl2)
    np.testing.assert_array_equal(nr, nr2)


@pytest.mark.parametrize("name", ["water192", "cu_cells5"])
def test_nlist_cells_equals_bruteforce(oracle_mod, name):
    w = synth.workload(name)
    o = oracle_mod.Oracle(synth.pack_blob(w["spec"]))
    a = o.nlist(w["coords"], w["types"], w["box"], use_cells=True)
    b = o.nlist(w["coords"], w["types"], w["box"], use_cells=False)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_fcc_shells_closed_form(oracle_mod):
    g = json.load(open(os.path.join(GOLD, "fcc_shells.json")))
    x, t, box = synth.fcc_copper(5, g["a"], jitter=0.0)
    spec = synth.copper_model(1)
    o = oracle_mod.Oracle(synth.pack_blob(spec))
    nl, nr, ovf = o.nlist(x, t, box)
    assert ovf == 0
    assert (nr[:, 0] == g["total_within_rcut"]).all()
    assert (nl[:, g["total_within_rcut"]:] == -1).all()
    radii = np.concatenate([[g["a"] * np.sqrt(n / 2.0)] * c for n, c in g["shells"]])
    for i in [0, 1, 77, 499]:
        d = x[nl[i, :176]] - x[i]
        d -= box * np.round(d / box)
        r = np.linalg.norm(d, axis=1)
        np.testing.assert_allclose(r, radii, rtol=0, atol=1e-9)   # sorted by distance, shell by shell
    # equal distances (a whole shell) are ordered by index
    d = x[nl[0, :12]] - x[0]
    assert np.all(np.diff(nl[0, :12]) > 0)


def test_nlist_overflow_keeps_nearest(oracle_mod):
    w = synth.workload("cu_cells5")
    full = synth.copper_model(1)
    small = synth.random_model(1, 8.0, 2.0, (40,), seed=1, desc_norm=8.0)
    of = oracle_mod.Oracle(synth.pack_blob(full))
    os_ = oracle_mod.Oracle(synth.pack_blob(small))
    a, ar, _ = of.nlist(w["coords"], w["types"], w["box"])
    b, br, ovf = os_.nlist(w["coords"], w["types"], w["box"])
    np.testing.assert_array_equal(b, a[:, :40])
    assert (br[:, 0] == 40).all()
    assert ovf == int((ar[:, 0] - 40).sum())


def test_nlist_rejects_small_box(oracle_mod):
    w = synth.workload("water192")
    o = oracle_mod.Oracle(synth.pack_blob(w["spec"]))
    with pytest.raises(ValueError):
        o.nlist(w["coords"], w["types"], np.array([11.9, 12.42, 12.42]))


# ---------------------------------------------------------------------------
# environment matrix: C2 switch, row identity, analytic Jacobian
# ---------------------------------------------------------------------------
def test_env_switch_and_row_identity(water):
    w, o = water
    rc, rcs = w["spec"].rcut, w["spec"].rcut_smth
    rhat = np.array([0.48, -0.6, 0.64])
    for r in [0.3, rcs * 0.999, 1.0, 3.0, 5.9]:
        R, _ = o.env_single(r * rhat)
        s = R[0]
        np.testing.assert_allclose(R @ R, 2 * s * s, rtol=1e-13)
        np.testing.assert_allclose(R[1:], s * rhat, rtol=1e-13)
        if r < rcs:
            np.testing.assert_allclose(s, 1.0 / r, rtol=1e-15)
    # sw = 1 at rcs; sw, sw', sw'' = 0 at rc (one-sided differences of r*s)
    sw = lambda r: o.env_single(r * rhat)[0][0] * r
    np.testing.assert_allclose(sw(rcs), 1.0, rtol=1e-15)
    assert sw(rc) == 0.0
    h = 1e-3
    assert abs(sw(rc - h)) < 20 * h ** 3
    assert abs((sw(rc - h) - sw(rc - 2 * h)) / h) < 60 * h ** 2
    assert abs((sw(rc) - 2 * sw(rc - h) + sw(rc - 2 * h)) / h ** 2) < 200 * h


def test_env_jacobian_fd(water):
    w, o = water
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=3)
        d *= rng.uniform(0.4, 5.9) / np.linalg.norm(d)
        _, J = o.env_single(d)
        h = 1e-6
        Jfd = np.empty((4, 3))
        for b in range(3):
            e = np.zeros(3)
            e[b] = h
            Jfd[:, b] = (o.env_single(d + e)[0] - o.env_single(d - e)[0]) / (2 * h)
        np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-8)


# ---------------------------------------------------------------------------
# descriptor: T and D computed a second way
# ---------------------------------------------------------------------------
def test_descriptor_pairwise_form(water):
    """D_ab = (1/Nc^2) sum_{j,k} G_ja G_kb (R_j . R_k): rotation invariant by
    construction; checks the contraction indices and the G< convention."""
    w, o = water
    spec = w["spec"]
    r = o.eval(w["coords"], w["types"], w["box"], intermediates=True)
    x = w["coords"] - w["box"] * np.floor(w["coords"] / w["box"])
    off = np.concatenate([[0], np.cumsum(spec.sel)])
    for i in [0, 1, 5, 100]:
        ti = w["types"][i]
        Gs, Rs = [], []
        for u in range(spec.ntypes):
            for p in range(r["nreal"][i, u]):
                j = r["nlist"][i, off[u] + p]
                d = x[j] - x[i]
                d -= w["box"] * np.round(d / w["box"])
                R, _ = o.env_single(d)
                Gs.append(o.embed(ti, u, R[0]))
                Rs.append(R)
        G, R = np.array(Gs), np.array(Rs)
        np.testing.assert_allclose(R, r["rt"][i][r["nlist"][i] >= 0], rtol=1e-12)
        Dpair = (G.T @ (R @ R.T) @ G[:, :spec.M2]) / spec.desc_norm ** 2
        np.testing.assert_allclose(r["D"][i].reshape(spec.M1, spec.M2), Dpair, rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(r["T"][i], G.T @ R / spec.desc_norm, rtol=1e-11, atol=1e-15)


# ---------------------------------------------------------------------------
# special cases with closed forms (weight surgery)
# ---------------------------------------------------------------------------
def _zero_emb(spec):
    for t in range(spec.ntypes):
        for u in range(spec.ntypes):
            for W in spec.emb_W[t][u]:
                W[:] = 0.0
    return spec


def test_embedding_closed_form_zero_weights(oracle_mod):
    """With all embedding weights zero, G is the bias cascade of the skip
    rule: 1->25 plain, 25->50 and 50->100 doubling (Fig. 1(e,f))."""
    spec = _zero_emb(synth.water_model(0))
    o = oracle_mod.Oracle(synth.pack_blob(spec))
    b = spec.emb_b[0][1]
    h1 = np.tanh(b[0])
    h2 = np.concatenate([h1, h1]) + np.tanh(b[1])
    h3 = np.concatenate([h2, h2]) + np.tanh(b[2])
    for s in [0.0, 0.3, 2.0]:
        np.testing.assert_allclose(o.embed(0, 1, s), h3, rtol=1e-13, atol=1e-15)


def test_embedding_student_shapes_skip_rule(oracle_mod):
    """Student widths 1->16->32->100: plain, doubling, plain."""
    spec = _zero_emb(synth.random_model(1, 8.0, 2.0, (64,), emb=(16, 32, 100), seed=3))
    o = oracle_mod.Oracle(synth.pack_blob(spec))
    b = spec.emb_b[0][0]
    h1 = np.tanh(b[0])
    h2 = np.concatenate([h1, h1]) + np.tanh(b[1])
    h3 = np.tanh(b[2])
    np.testing.assert_allclose(o.embed(0, 0, 0.7), h3, rtol=1e-13, atol=1e-15)


def test_fitting_closed_form(oracle_mod):
    """Zero the fitting weights of layers 1..3: x1 = tanh(b1) and the two
    identity-skip layers add tanh(b2), tanh(b3) (Fig. 1(g)); E_i is
    (x1 + tanh b2 + tanh b3) . W4 + b4 for every atom, so forces vanish."""
    w = synth.workload("water192")
    spec = w["spec"]
    for t in range(spec.ntypes):
        for W in spec.fit_W[t][:3]:
            W[:] = 0.0
    o = oracle_mod.Oracle(synth.pack_blob(spec))
    r = o.eval(w["coords"], w["types"], w["box"])
    for t in range(spec.ntypes):
        b = spec.fit_b[t]
        x = np.tanh(b[0]) + np.tanh(b[1]) + np.tanh(b[2])
        e = x @ spec.fit_W[t][3][:, 0] + b[3][0]
        np.testing.assert_allclose(r["atom_e"][w["types"] == t], e, rtol=1e-14)
    assert np.abs(r["force"]).max() < 1e-12


def test_dimer_closed_form(oracle_mod):
    """Two atoms: D = (2 s^2 / Nc^2) G G<^T; F = -E'(r) r_hat; Xi = -g (x) d."""
    spec = synth.water_model(0)
    o = oracle_mod.Oracle(synth.pack_blob(spec))
    box = np.full(3, 20.0)
    rhat = np.array([2.0, -1.0, 2.0]) / 3.0
    types = np.array([0, 1], dtype=np.int32)

    def E(r):
        x = np.array([[5.0, 5.0, 5.0], 5.0 + r * rhat])
        return o.eval(x, types, box, intermediates=True)

    r0 = 1.7
    res = E(r0)
    R, _ = o.env_single(r0 * rhat)
    s = R[0]
    for i, (ti, u) in enumerate([(0, 1), (1, 0)]):
        G = o.embed(ti, u, s)
        Dc = 2 * s * s / spec.desc_norm ** 2 * np.outer(G, G[:spec.M2])
        np.testing.assert_allclose(res["D"][i].reshape(spec.M1, spec.M2), Dc, rtol=1e-12)
    h = 1e-5
    dE = (E(r0 + h)["energy"] - E(r0 - h)["energy"]) / (2 * h)
    np.testing.assert_allclose(res["force"][1], -dE * rhat, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(res["force"][0], dE * rhat, rtol=1e-7, atol=1e-9)
    # virial: g = dE/dd = dE * rhat, d = r0 * rhat
    np.testing.assert_allclose(res["virial"], -np.outer(dE * rhat, r0 * rhat), rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------------------
# forces and virial by finite differences
# ---------------------------------------------------------------------------
def _local_fd_force(o, x, types, box, k, nl_full, h=1e-5):
    """Central difference of the local energy sum_{i in {k} + N(k)} E_i."""
    cen = np.unique(np.concatenate([[k], nl_full[k][nl_full[k] >= 0]]))
    f = np.empty(3)
    for a in range(3):
        xp, xm = x.copy(), x.copy()
        xp[k, a] += h
        xm[k, a] -= h
        rp = o.eval(xp, types, box, centres=cen)
        em = o.eval(xm, types, box, centres=cen)["energy"]
        f[a] = -(rp["energy"] - em) / (2 * h)
    # rounding bound of the difference quotient: a few ulps of sum |E_i|
    tol = 8 * np.finfo(float).eps * np.abs(rp["atom_e"]).sum() / (2 * h)
    return f, max(tol, 1e-8)


@pytest.mark.parametrize("name", ["water192", "cu_cells5"])
def test_forces_central_fd(oracle_mod, name):
    w = synth.workload(name)
    o = oracle_mod.Oracle(synth.pack_blob(w["spec"]))
    x, t, box = w["coords"], w["types"], w["box"]
    r = o.eval(x, t, box)
    nl, _, _ = o.nlist(x, t, box)
    rng = np.random.default_rng(7)
    for k in rng.choice(len(t), size=6, replace=False):
        fd, tol = _local_fd_force(o, x, t, box, k, nl)
        assert tol < 1e-6
        np.testing.assert_allclose(r["force"][k], fd, rtol=0, atol=tol)


def test_forces_central_fd_wide_net(oracle_mod):
    """A net of the embedding-size study (128-256-512: D has 8,192 features,
    more than the oracle's former per-layer scratch) on 108 disordered
    copper atoms, rc 4.5 A: forces equal central differences of the energy."""
    x, t, box = synth.fcc_copper(3, 3.634, 0.25, seed=7)
    spec = synth.random_model(1, 4.5, 1.0, (64,), emb=(128, 256, 512), seed=21)
    o = oracle_mod.Oracle(synth.pack_blob(spec))
    r = o.eval(x, t, box)
    nl, _, _ = o.nlist(x, t, box)
    for k in np.random.default_rng(8).choice(len(t), size=3, replace=False):
        fd, tol = _local_fd_force(o, x, t, box, k, nl)
        assert tol < 1e-6
        np.testing.assert_allclose(r["force"][k], fd, rtol=0, atol=tol)


def test_total_energy_fd_and_force_sum(water):
    w, o = water
    x, t, box = w["coords"], w["types"], w["box"]
    r = o.eval(x, t, box)
    f = r["force"]
    rms = np.sqrt((f ** 2).sum(1).mean())
    assert np.abs(f.sum(0)).max() <= 1e-10 * rms * np.sqrt(len(t))
    k, a, h = 17, 1, 1e-5
    xp, xm = x.copy(), x.copy()
    xp[k, a] += h
    xm[k, a] -= h
    fd = -(o.eval(xp, t, box)["energy"] - o.eval(xm, t, box)["energy"]) / (2 * h)
    assert abs(fd - f[k, a]) < 1e-5


def test_virial_diagonal_strain_fd(water):
    w, o = water
    x, t, box = w["coords"], w["types"], w["box"]
    r = o.eval(x, t, box)
    h = 1e-6
    for a in range(3):
        s = np.ones(3)
        s[a] += h
        ep = o.eval(x * s, t, box * s)["energy"]
        s[a] -= 2 * h
        em = o.eval(x * s, t, box * s)["energy"]
        dE = (ep - em) / (2 * h)
        np.testing.assert_allclose(r["virial"][a, a], -dE, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(r["virial"], r["virial"].T, rtol=1e-10, atol=1e-10)


def _cluster(w, radius):
    x = w["coords"]
    c = x.mean(0)
    keep = np.linalg.norm(x - c, axis=1) < radius
    box = np.full(3, 60.0)
    return x[keep] - c + 30.0, w["types"][keep], box


def test_virial_full_tensor_isolated_cluster(water):
    """Off-diagonal elements: homogeneous strain x -> (I + eps) x of an
    isolated cluster (periodic images far beyond the cutoff)."""
    w, o = water
    x, t, box = _cluster(w, 5.5)
    c = np.full(3, 30.0)
    r = o.eval(x, t, box)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            ep = o.eval(c + (x - c) @ (np.eye(3) + e).T, t, box)["energy"]
            em = o.eval(c + (x - c) @ (np.eye(3) - e).T, t, box)["energy"]
            np.testing.assert_allclose(r["virial"][a, b], -(ep - em) / (2 * h), rtol=1e-6, atol=1e-6)


# ---------------------------------------------------------------------------
# invariances
# ---------------------------------------------------------------------------
def test_translation_and_permutation_invariance(water):
    w, o = water
    x, t, box = w["coords"], w["types"], w["box"]
    r = o.eval(x, t, box)
    r2 = o.eval(x + np.array([3.3, -7.1, 100.25]), t, box)
    np.testing.assert_allclose(r2["energy"], r["energy"], rtol=1e-12)
    np.testing.assert_allclose(r2["force"], r["force"], rtol=0, atol=1e-10)
    rng = np.random.default_rng(3)
    perm = np.arange(len(t))
    for ty in (0, 1):
        idx = np.nonzero(t == ty)[0]
        perm[idx] = rng.permutation(idx)
    r3 = o.eval(x[perm], t[perm], box)
    np.testing.assert_allclose(r3["energy"], r["energy"], rtol=1e-12)
    np.testing.assert_allclose(r3["force"], r["force"][perm], rtol=0, atol=1e-10)


def test_rotation_invariance_cluster(water):
    w, o = water
    x, t, box = _cluster(w, 6.0)
    c = np.full(3, 30.0)
    r = o.eval(x, t, box)
    Q = synth._random_rotation(np.random.default_rng(11))
    r2 = o.eval(c + (x - c) @ Q.T, t, box)
    np.testing.assert_allclose(r2["energy"], r["energy"], rtol=1e-12)
    np.testing.assert_allclose(r2["force"], r["force"] @ Q.T, rtol=0, atol=1e-10)


def test_cubic_symmetry_periodic(water):
    w, o = water
    x, t, box = w["coords"], w["types"], w["box"]
    r = o.eval(x, t, box)
    L = box[0]
    x2 = x[:, [2, 0, 1]].copy()      # axis permutation
    x2[:, 1] = L - x2[:, 1]          # reflection
    r2 = o.eval(x2, t, box)
    np.testing.assert_allclose(r2["energy"], r["energy"], rtol=1e-12)


def test_smooth_at_cutoff(water):
    """An atom crossing rc radially: E continuous, jump O(delta^3)."""
    w, o = water
    spec = w["spec"]
    box = np.full(3, 20.0)
    t = np.array([0, 1], dtype=np.int32)
    rhat = np.array([0.0, 0.6, 0.8])
    E = lambda r: o.eval(np.array([[5.0] * 3, 5.0 + r * rhat]), t, box)["energy"]
    e_far = E(spec.rcut + 0.5)
    for dlt in [1e-2, 1e-3]:
        assert abs(E(spec.rcut - dlt) - e_far) < 1e4 * dlt ** 3
    assert E(spec.rcut) == e_far


# ---------------------------------------------------------------------------
# velocity Verlet
# ---------------------------------------------------------------------------
def test_verlet_reversible_and_dt2(water):
    w, o = water
    x, t, box, m = w["coords"], w["types"], w["box"], w["masses"]
    v = synth.maxwell_boltzmann(m[t], 300.0, 1)
    n = 10
    x1, v1, th = o.verlet(x, v, t, box, m, 0.5, n)
    x2, v2, _ = o.verlet(x1, -v1, t, box, m, 0.5, n)
    d = x2 - x
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-v2, v, rtol=0, atol=1e-9)
    # energy fluctuation shrinks ~4x when dt halves over the same time
    _, _, tha = o.verlet(x, v, t, box, m, 0.5, 10)
    _, _, thb = o.verlet(x, v, t, box, m, 0.25, 20)
    fa = np.ptp(tha[:, 3])
    fb = np.ptp(thb[:, 3])
    assert 3.0 < fa / fb < 5.0


def test_maxwell_boltzmann_exact_temperature():
    m = np.full(300, 63.546)
    v = synth.maxwell_boltzmann(m, 300.0, 5)
    ke = 0.5 * synth.MVV2E * (m[:, None] * v * v).sum()
    np.testing.assert_allclose(2 * ke / ((3 * 300 - 3) * synth.KB_EV), 300.0, rtol=1e-12)
    np.testing.assert_allclose((m[:, None] * v).sum(0), 0.0, atol=1e-12)


# ---------------------------------------------------------------------------
# MD units and thermo columns (Section VI: NVE runs in metal units, thermo
# output of kinetic, potential and total energy, temperature and pressure).
# The conversion factors below are derived here from the SI definitions
# (CODATA 2018: e and k_B exact, the atomic mass constant measured), not
# taken from the oracle or the structure generator.
# ---------------------------------------------------------------------------
_E_CHARGE = 1.602176634e-19      # J per eV (exact)
_K_BOLTZ = 1.380649e-23          # J/K (exact)
_AMU = 1.66053906660e-27         # kg
_MVV2E_SI = _AMU * (1e-10 / 1e-15) ** 2 / _E_CHARGE     # amu A^2/fs^2 -> eV
_ACC_SI = _E_CHARGE / 1e-10 / _AMU * 1e-15 ** 2 / 1e-10  # eV/(A amu) -> A/fs^2
_KB_SI = _K_BOLTZ / _E_CHARGE                             # eV/K


def _zero_force_model():
    """Water model with the output weights zeroed: E_i = b4 = 0 for every
    atom, so forces and virial vanish (weight surgery, Fig. 1(g))."""
    spec = synth.water_model(0)
    for t in range(spec.ntypes):
        spec.fit_W[t][3][:] = 0.0
        spec.fit_b[t][3][:] = 0.0
    return spec


def test_md_unit_constants_from_si():
    """The two conversions the integrator needs, written out from SI."""
    np.testing.assert_allclose(_MVV2E_SI, 103.6427, rtol=1e-6)
    np.testing.assert_allclose(_ACC_SI, 9.648533212e-3, rtol=1e-9)
    np.testing.assert_allclose(_ACC_SI * _MVV2E_SI, 1.0, rtol=1e-12)
    np.testing.assert_allclose(_KB_SI, 8.617333262e-5, rtol=1e-9)


def test_thermo_kinetic_temperature_ideal_gas(oracle_mod):
    """Zero-force model, 0 steps: thermo row 0 holds KE = sum m v^2 / 2 in
    eV, T from equipartition over 3N - 3 degrees of freedom, and the ideal
    gas pressure P V = 2 KE / 3 = (N - 1) k_B T (no virial term)."""
    w = synth.workload("water192")
    o = oracle_mod.Oracle(synth.pack_blob(_zero_force_model()))
    t = w["types"]
    n = len(t)
    rng = np.random.default_rng(11)
    v = rng.normal(scale=0.01, size=(n, 3))          # A/fs, arbitrary
    m = w["masses"][t]
    _, _, th = o.verlet(w["coords"], v, t, w["box"], w["masses"], 0.5, 0, every=1)
    ke = 0.5 * (m[:, None] * v * v).sum() * _MVV2E_SI
    vol = float(np.prod(w["box"]))
    np.testing.assert_allclose(th[0, 1], ke, rtol=1e-9)
    np.testing.assert_allclose(th[0, 2], 0.0, atol=1e-12)
    np.testing.assert_allclose(th[0, 3], ke, rtol=1e-9)
    np.testing.assert_allclose(th[0, 4], 2 * ke / ((3 * n - 3) * _KB_SI), rtol=1e-9)
    np.testing.assert_allclose(th[0, 5] * vol, (n - 1) * _KB_SI * th[0, 4], rtol=1e-9)
    np.testing.assert_allclose(th[0, 5] * vol, 2 * ke / 3, rtol=1e-9)


def test_verlet_free_flight_and_kick_units(oracle_mod):
    """Free flight: with zero forces x advances by dt v per step and v
    stays.  Kick: a dimer released at rest moves, after one step, to
    x0 + dt^2 F0/(2m) and has v = dt (F0 + F1)/(2m), with the force-to-
    acceleration factor from SI."""
    w = synth.workload("water192")
    o0 = oracle_mod.Oracle(synth.pack_blob(_zero_force_model()))
    t, box = w["types"], w["box"]
    rng = np.random.default_rng(12)
    v = rng.normal(scale=0.01, size=(len(t), 3))
    x1, v1, _ = o0.verlet(w["coords"], v, t, box, w["masses"], 0.5, 4, every=4)
    d = x1 - (w["coords"] + 4 * 0.5 * v)
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-12
    np.testing.assert_array_equal(v1, v)

    spec = synth.water_model(0)
    o = oracle_mod.Oracle(synth.pack_blob(spec))
    boxd = np.full(3, 20.0)
    types = np.array([0, 1], dtype=np.int32)
    x0 = np.array([[5.0, 5.0, 5.0], [6.0, 5.5, 4.2]])
    masses = np.array([synth.MASS["O"], synth.MASS["H"]])
    dt = 0.5
    f0 = o.eval(x0, types, boxd)["force"]
    xe = x0 + 0.5 * dt * dt * f0 / masses[types][:, None] * _ACC_SI
    f1 = o.eval(xe, types, boxd)["force"]
    ve = 0.5 * dt * (f0 + f1) / masses[types][:, None] * _ACC_SI
    xs, vs, _ = o.verlet(x0, np.zeros((2, 3)), types, boxd, masses, dt, 1, every=1)
    assert np.abs(f0).max() > 1e-2        # the kick is not vacuous
    np.testing.assert_allclose(xs, xe, rtol=0, atol=1e-13)
    np.testing.assert_allclose(vs, ve, rtol=1e-9, atol=1e-15)


def test_thermo_pressure_is_minus_dE_dV(oracle_mod):
    """At rest the pressure column is the configurational pressure
    -dE/dV under isotropic scaling of the box and all positions (central
    difference of the energy); with velocities it adds 2 KE / (3 V)."""
    w = synth.workload("water192")
    o = oracle_mod.Oracle(synth.pack_blob(w["spec"]))
    x, t, box = w["coords"], w["types"], w["box"]
    _, _, th = o.verlet(x, np.zeros_like(x), t, box, w["masses"], 0.5, 0, every=1)
    eps = 1e-5
    e = []
    for sgn in (1, -1):
        s = 1 + sgn * eps
        e.append(o.eval(x * s, t, box * s)["energy"])
    vol = float(np.prod(box))
    dV = vol * ((1 + eps) ** 3 - (1 - eps) ** 3)
    p_fd = -(e[0] - e[1]) / dV
    assert abs(p_fd) > 1e-4
    np.testing.assert_allclose(th[0, 5], p_fd, rtol=1e-6)
    np.testing.assert_allclose(th[0, 1], 0.0, atol=0)
    # with velocities: P = (2 KE + tr Xi) / (3 V), the two parts pinned apart
    rng = np.random.default_rng(13)
    v = rng.normal(scale=0.01, size=x.shape)
    _, _, thv = o.verlet(x, v, t, box, w["masses"], 0.5, 0, every=1)
    ke = 0.5 * (w["masses"][t][:, None] * v * v).sum() * _MVV2E_SI
    np.testing.assert_allclose(thv[0, 5], p_fd + 2 * ke / (3 * vol), rtol=1e-6)
