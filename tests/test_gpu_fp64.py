"""Parity of the FP64 HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: neighbour list bit-exact; energy within 1e-10 relative; forces within
1e-9 eV/A absolute; virial within 1e-10 relative to its largest element.
Full-size workloads are checked on sampled atoms the oracle evaluates one by
one (local environments), plus size-independent properties."""
import sys

import numpy as np
import pytest

from paper_2005_00223_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_cache = {}


def work(name):
    if name not in _cache:
        if name == "fcc_perfect5":
            x, t, box = synth.fcc_copper(5, 3.634, jitter=0.0)
            w = dict(name=name, coords=x, types=t, box=box, spec=synth.copper_model(1),
                     masses=np.array([synth.MASS["Cu"]]))
        elif name == "water191":
            w = dict(synth.workload("water192"))
            keep = np.arange(192) != 77
            w.update(name=name, coords=w["coords"][keep], types=w["types"][keep])
        else:
            w = synth.workload(name)
        w["blob"] = synth.pack_blob(w["spec"])
        _cache[name] = w
    return _cache[name]


def gpu_model(w):
    from paper_2005_00223_amd.model import DPModel
    return DPModel(w["blob"], "fp64")


def oracle(w):
    from oracle import oracle as O
    return O.Oracle(w["blob"])


def f_tol(a, b, tol):
    err = np.abs(np.asarray(a) - np.asarray(b)).max()
    assert err <= tol, f"max abs error {err:.3e} > {tol:.1e}"


def rel_tol(a, b, tol):
    a, b = np.asarray(a), np.asarray(b)
    err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    assert err <= tol, f"relative error {err:.3e} > {tol:.1e}"


@pytest.mark.parametrize("name", ["water192", "water191", "cu_cells5", "fcc_perfect5", "water12288"])
def test_nlist_bit_exact(name):
    w = work(name)
    say(f"[nlist] {name} n={len(w['types'])}")
    m = gpu_model(w)
    n = len(w["types"])
    m.compute(w["coords"], w["types"], w["box"])
    nl, nr = m.nlist(n, w["spec"].nnei, w["spec"].ntypes)
    onl, onr, ovf = oracle(w).nlist(w["coords"], w["types"], w["box"])
    np.testing.assert_array_equal(nl.cpu().numpy(), onl)
    np.testing.assert_array_equal(nr.cpu().numpy(), onr)
    st = m.stats()
    assert st["sel_overflow"] == ovf
    assert st["max_real"][: w["spec"].ntypes] == list(onr.max(0)) or ovf > 0


@pytest.mark.parametrize("name", ["water192", "water191", "cu_cells5", "water12288"])
def test_energy_force_virial(name):
    w = work(name)
    say(f"[efv] {name} n={len(w['types'])}")
    m = gpu_model(w)
    e, f, v = m.compute(w["coords"], w["types"], w["box"])
    r = oracle(w).eval(w["coords"], w["types"], w["box"])
    rel_tol(e.item(), r["energy"], 1e-10)
    f_tol(f.cpu().numpy(), r["force"], 1e-9)
    rel_tol(v.cpu().numpy(), r["virial"], 1e-10)


def test_intermediates_water192():
    w = work("water192")
    say("[intermediates] water192")
    spec = w["spec"]
    n = len(w["types"])
    m = gpu_model(w)
    m.compute(w["coords"], w["types"], w["box"], keep_intermediates=True)
    g = {k: v.cpu().numpy() for k, v in m.intermediates(n, spec.M1, spec.M2, spec.nnei).items()}
    r = oracle(w).eval(w["coords"], w["types"], w["box"], intermediates=True)
    rel_tol(g["atom_e"], r["atom_e"], 1e-12)
    rel_tol(g["T"], r["T"], 1e-12)
    rel_tol(g["D"], r["D"], 1e-12)
    real = r["nlist"] >= 0
    rel_tol(g["net_deriv"][real], r["net_deriv"][real], 1e-11)


def _sampled_check(w, m, n_sample, seed, f_bar=1e-9):
    """Forces of sampled atoms against one oracle evaluation whose centres
    are the sampled atoms and all their neighbours: the force on k depends
    only on the energies of k and of the atoms within rc of it (the list
    relation is symmetric when no type overflows its sel), so those forces
    are exact; per-atom energies of the sampled atoms."""
    o = oracle(w)
    n = len(w["types"])
    spec = w["spec"]
    rng = np.random.default_rng(seed)
    ks = np.sort(rng.choice(n, size=n_sample, replace=False))
    e, f, v = m.compute(w["coords"], w["types"], w["box"], keep_intermediates=False)
    f = f.cpu().numpy()
    vv = v.cpu().numpy()
    nl, _ = m.nlist(n, spec.nnei, spec.ntypes)
    nl = nl.cpu().numpy()
    assert m.stats()["sel_overflow"] == 0
    ae = m.intermediates(n, spec.M1, spec.M2, spec.nnei, which=("atom_e",))["atom_e"].cpu().numpy()
    onl, _, _ = o.nlist(w["coords"], w["types"], w["box"], centres=ks)
    np.testing.assert_array_equal(nl[ks], onl)
    cen = np.unique(np.concatenate([ks, nl[ks][nl[ks] >= 0]]))
    say(f"  {n_sample} sampled atoms, {cen.size} oracle centres")
    r = o.eval(w["coords"], w["types"], w["box"], centres=cen)
    f_tol(f[ks], r["force"][ks], f_bar)
    rel_tol(ae[ks], r["atom_e"][np.searchsorted(cen, ks)], 1e-10)
    # size-independent properties: sum of forces, symmetric virial
    rms = np.sqrt((f ** 2).sum(1).mean())
    assert np.abs(f.sum(0)).max() <= 1e-9 * rms * np.sqrt(n)
    rel_tol(vv, vv.T, 1e-10)
    return e.item()


def test_cu32000_sampled():
    w = work("cu32000")
    say("[sampled] cu32000")
    _sampled_check(w, gpu_model(w), 64, 0)


def test_cu500k_sampled():
    """The benchmark workload at full size (500,000 atoms) in the same
    single-evaluation launch configuration the benchmark's MD step uses."""
    w = work("cu500k")
    say("[sampled] cu500k")
    _sampled_check(w, gpu_model(w), 256, 1)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_empty_system():
    w = work("water192")
    say("[edge] empty")
    m = gpu_model(w)
    e, f, v = m.compute(np.zeros((0, 3)), np.zeros(0, dtype=np.int32), w["box"])
    assert e.item() == 0.0 and f.shape == (0, 3)
    assert np.all(v.cpu().numpy() == 0.0)


def test_isolated_atoms_and_single_type():
    w = work("water192")
    say("[edge] isolated")
    box = np.full(3, 30.0)
    x = np.array([[1.0, 1.0, 1.0], [15.0, 15.0, 15.0], [15.9, 15.2, 14.8], [1.5, 28.9, 1.2]])
    t = np.array([1, 1, 1, 1], dtype=np.int32)
    m = gpu_model(w)
    e, f, v = m.compute(x, t, box)
    r = oracle(w).eval(x, t, box)
    rel_tol(e.item(), r["energy"], 1e-12)
    f_tol(f.cpu().numpy(), r["force"], 1e-9)


def test_sel_overflow_keeps_nearest():
    say("[edge] overflow")
    w = dict(work("cu_cells5"))
    spec = synth.random_model(1, 8.0, 2.0, (40,), seed=1, desc_norm=8.0, out_scale=50.0)
    w["blob"] = synth.pack_blob(spec)
    w["spec"] = spec
    m = gpu_model(w)
    e, f, v = m.compute(w["coords"], w["types"], w["box"])
    nl, _ = m.nlist(len(w["types"]), 40, 1)
    o = oracle(w)
    onl, _, ovf = o.nlist(w["coords"], w["types"], w["box"])
    np.testing.assert_array_equal(nl.cpu().numpy(), onl)
    assert m.stats()["sel_overflow"] == ovf > 0
    r = o.eval(w["coords"], w["types"], w["box"])
    rel_tol(e.item(), r["energy"], 1e-10)
    f_tol(f.cpu().numpy(), r["force"], 1e-9)


def test_errors_are_reported():
    from paper_2005_00223_amd import _lib
    w = work("water192")
    say("[edge] errors")
    m = gpu_model(w)
    bad = w["types"].copy()
    bad[5] = 7
    with pytest.raises(_lib.DPError) as ei:
        m.compute(w["coords"], bad, w["box"])
    assert ei.value.code == _lib.DP_E_TYPE
    with pytest.raises(_lib.DPError) as ei:
        m.compute(w["coords"], w["types"], np.array([11.9, 12.42, 12.42]))
    assert ei.value.code == _lib.DP_E_BOX
    tri = np.diag(w["box"]).astype(float)
    tri[0, 1] = 0.5
    with pytest.raises(_lib.DPError) as ei:
        m.compute(w["coords"], w["types"], tri)
    assert ei.value.code == _lib.DP_E_BOX
    # a good call afterwards still works
    e, f, v = m.compute(w["coords"], w["types"], w["box"])
    assert np.isfinite(e.item())


def test_deterministic_nlist_and_energy():
    w = work("water12288")
    say("[determinism] water12288")
    m = gpu_model(w)
    n = len(w["types"])
    e1, f1, _ = m.compute(w["coords"], w["types"], w["box"])
    nl1, _ = m.nlist(n, w["spec"].nnei, w["spec"].ntypes)
    e2, f2, _ = m.compute(w["coords"], w["types"], w["box"])
    nl2, _ = m.nlist(n, w["spec"].nnei, w["spec"].ntypes)
    assert torch.equal(nl1, nl2)
    assert e1.item() == e2.item()   # fixed-order energy reduction
    f_tol(f1.cpu().numpy(), f2.cpu().numpy(), 1e-12)


# ---------------------------------------------------------------------------
# MD driver
# ---------------------------------------------------------------------------
def test_md_resume_equals_continuous_run():
    """Checkpoint / resume: the MD state is the caller's (x, v); 10 steps,
    then 10 more from the returned arrays, equal 20 steps in one call (the
    list is rebuilt at the start of each call; the FP64 forces do not depend
    on the candidate list, only their atomic summation order may differ)."""
    w = work("water192")
    say("[md] resume water192 10 + 10 steps")
    t = w["types"]
    v0 = synth.maxwell_boltzmann(w["masses"][t], 300.0, w["vseed"])
    m = gpu_model(w)
    runs = []
    for parts in ((20,), (10, 10)):
        x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda")
        v = torch.tensor(v0, dtype=torch.float64, device="cuda")
        for k in parts:
            m.md_run(x, v, t, w["box"], w["masses"], 0.5, k, skin=0.2, thermo_every=k)
        runs.append((x.cpu().numpy(), v.cpu().numpy()))
    d = runs[0][0] - runs[1][0]
    d -= w["box"] * np.round(d / w["box"])
    say(f"  max |dx| {np.abs(d).max():.2e}, max |dv| {np.abs(runs[0][1] - runs[1][1]).max():.2e}")
    assert np.abs(d).max() < 1e-11
    assert np.abs(runs[0][1] - runs[1][1]).max() < 1e-11


def test_md_matches_oracle_verlet():
    w = work("water192")
    say("[md] water192 20 steps")
    t = w["types"]
    v0 = synth.maxwell_boltzmann(w["masses"][t], 300.0, w["vseed"])
    m = gpu_model(w)
    x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda")
    v = torch.tensor(v0, dtype=torch.float64, device="cuda")
    th = m.md_run(x, v, t, w["box"], w["masses"], 0.5, 20, skin=0.2, thermo_every=5)
    ox, ov, oth = oracle(w).verlet(w["coords"], v0, t, w["box"], w["masses"], 0.5, 20, every=5)
    d = x.cpu().numpy() - ox
    d -= w["box"] * np.round(d / w["box"])
    assert np.abs(d).max() < 1e-9
    f_tol(v.cpu().numpy(), ov, 1e-9)
    thg = th.cpu().numpy()
    # all six columns: step, KE, PE, KE + PE, T, P (P carries the virial)
    np.testing.assert_array_equal(thg[:, 0], oth[:, 0])
    for c in range(1, 6):
        rel_tol(thg[:, c], oth[:, c], 1e-9)


def test_md_regrows_an_overflowing_candidate_list():
    """256 copper atoms (4^3 FCC cells) in the middle of a box twice as
    wide: the candidate capacity sized from the mean density (128 per atom)
    overflows on the first list build.  The run stops on the device at that
    step, grows the list, resumes, and ends where a run with the grown list
    from the start ends."""
    say("[md] candidate list regrowth")
    x0, t, box = synth.fcc_copper(4, 3.634, jitter=0.05, seed=9)
    box2 = 2.0 * np.asarray(box, dtype=np.float64)
    x0 = x0 + 0.25 * box2
    spec = synth.copper_model(1)
    w = dict(coords=x0, types=t, box=box2, spec=spec, blob=synth.pack_blob(spec),
             masses=np.array([synth.MASS["Cu"]]))
    v0 = synth.maxwell_boltzmann(w["masses"][t], 300.0, 109)

    def run(m):
        x = torch.tensor(x0, dtype=torch.float64, device="cuda")
        v = torch.tensor(v0, dtype=torch.float64, device="cuda")
        th = m.md_run(x, v, t, box2, w["masses"], 1.0, 20, skin=1.0, thermo_every=10)
        return x.cpu().numpy(), v.cpu().numpy(), th.cpu().numpy()

    a = gpu_model(w)
    xa, va, tha = run(a)
    st = a.stats()
    say(f"  candidate capacity after the run: {st['cand_cap']}")
    assert st["cand_cap"] >= 256
    b = gpu_model(w)
    xx = torch.tensor(x0, dtype=torch.float64, device="cuda")
    vv = torch.tensor(v0, dtype=torch.float64, device="cuda")
    b.md_run(xx, vv, t, box2, w["masses"], 1.0, 1, skin=1.0, thermo_every=1)  # grows b's list
    xb, vb, thb = run(b)
    assert np.all(np.isfinite(tha))
    f_tol(xa, xb, 1e-9)
    f_tol(va, vb, 1e-9)
    rel_tol(tha, thb, 1e-9)
