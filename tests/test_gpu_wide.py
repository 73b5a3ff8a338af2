"""Wide embedding nets (the embedding-size study of Sec. VII-D, Fig. 7)
through the 16-bit GEMM path, against the FP64 oracle.

The oracle runs the same model with its 16-bit weights rounded beforehand
(GEMM layers of the embedding nets, the first two fitting layers), so the
difference left is the path's own: activations and their tangents stored
between layers either as one 16-bit value (the paper's MIX-16 storage) or as
hi + lo 16-bit halves (the default), FP32 GEMM accumulation and FP32 sums
of T.  Cases: the study's smallest matrix
(64 x 128, net 32-64-128, on the register-resident kernels), the smallest
wide net
(64-128-256) in FP16 and BF16, 256-512-1024, the largest net of the study
(512-1024-2048), and two atom types (four nets, one GEMM row block each).
The full-size sweep workload (13,500 copper atoms, rc 8 A) is checked on the
per-atom energies of sampled atoms, which the oracle evaluates centre by
centre."""
import copy
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


def _quantised(spec, prec):
    """The model with the weights the 16-bit kernels hold, in FP64."""
    from oracle import student as S
    q = copy.deepcopy(spec)
    p = 0 if prec == "fp16" else 1
    for t in range(spec.ntypes):
        for u in range(spec.ntypes):
            for l in range(1, len(spec.emb)):
                q.emb_W[t][u][l] = S.round16(spec.emb_W[t][u][l], p)
        for l in range(2):
            q.fit_W[t][l] = S.round16(spec.fit_W[t][l], p)
    return q


def _system(name):
    if name == "cu3":  # 3^3 FCC cells, 108 atoms, 10.9 A box, strongly disordered
        return synth.fcc_copper(3, 3.634, 0.25, seed=7)
    w = synth.workload(name)
    return w["coords"], w["types"], w["box"]


def _model(name, rc, emb, seed=21):
    if name == "cu3":
        return synth.random_model(1, rc, 1.0, (64,), emb=emb, seed=seed)
    return synth.random_model(2, rc, 0.5, (46, 92), emb=emb, seed=seed)


# relative force RMSE, relative energy, relative virial bars per precision:
# 16-bit storage of every activation and tangent (unit roundoff u = 2^-11
# FP16, 2^-8 BF16) leaves a few u of relative error per feature, and the
# forces carry it at about 2u (measured); the bars are 10u for forces and
# the virial.  Energies are dominated by the fitting biases and agree far
# better; their bars are u/5.
BARS = {"fp16": (5e-3, 1e-4, 5e-3), "bf16": (4e-2, 8e-4, 4e-2)}
# split storage (hi + lo halves, two products): the activations carry ~2^-22
# (FP16) / ~2^-16 (BF16) relative; what remains in the forces is FP32
# accumulation, ~1e-5 (measured 3e-6 - 1.4e-5): bars 2e-4 / 1e-3.  Energies
# are limited by the fitting net's arithmetic, as with either storage.
BARS_SPLIT = {"fp16": (2e-4, 1e-4, 2e-4), "bf16": (1e-3, 8e-4, 1e-3)}


@pytest.mark.parametrize("sysname,rc,emb,prec,storage", [
    ("cu3", 4.5, (32, 64, 128), "fp16", "split"),
    ("cu3", 4.5, (64, 128, 256), "fp16", "mix16"),
    ("cu3", 4.5, (64, 128, 256), "fp16", "split"),
    ("cu3", 4.5, (64, 128, 256), "bf16", "mix16"),
    ("cu3", 4.5, (64, 128, 256), "bf16", "split"),
    ("cu3", 4.5, (256, 512, 1024), "fp16", "mix16"),
    ("cu3", 4.5, (256, 512, 1024), "fp16", "split"),
    ("cu3", 3.7, (512, 1024, 2048), "fp16", "mix16"),
    ("cu3", 3.7, (512, 1024, 2048), "fp16", "split"),
    # M1 = 1280: 160 feature columns per T workgroup, which does not divide
    # its 256 threads (the threads past 160 must stay idle)
    ("cu3", 3.7, (320, 640, 1280), "fp16", "mix16"),
    ("cu3", 3.7, (320, 640, 1280), "fp16", "split"),
    ("water192", 6.0, (64, 128, 256), "fp16", "mix16"),
    ("water192", 6.0, (64, 128, 256), "fp16", "split"),
])
def test_wide_matches_oracle(sysname, rc, emb, prec, storage):
    from oracle import oracle as O
    from paper_2005_00223_amd.model import DPModel
    x, t, box = _system(sysname)
    spec = _model(sysname, rc, emb)
    say(f"[wide] {sysname} rc {rc} emb {emb} {prec} {storage}: {len(t)} atoms")
    m = DPModel(synth.pack_blob(spec), prec)
    m.set_wide_storage(0 if storage == "split" else 1)
    e, f, v = m.compute(x, t, box)
    st = m.stats()
    # 32-64-128 runs the register-resident kernels (hi/lo split activations)
    assert st["wide_evals"] == (0 if emb[-1] <= 128 else 1)
    f = f.cpu().numpy()
    v = np.asarray(v.cpu().numpy()).reshape(-1)
    r = O.Oracle(synth.pack_blob(_quantised(spec, prec))).eval(x, t, box)
    rms = float(np.sqrt((r["force"] ** 2).sum(1).mean()))
    df = float(np.sqrt(((f - r["force"]) ** 2).sum(1).mean()))
    de = abs(float(e) - r["energy"])
    vo = np.asarray(r["virial"]).reshape(-1)
    dv = float(np.abs(v - vo).max())
    vs = max(1e-12, float(np.abs(vo).max()))
    say(f"  force RMSE {df:.3e} (RMS|F| {rms:.3e}, rel {df / rms:.2e}), |dE| {de:.3e} "
        f"(E {r['energy']:.4e}, rel {de / abs(r['energy']):.2e}), max|dV| {dv:.3e} (rel {dv / vs:.2e})")
    # nets up to 128 wide run the register-resident kernels whatever the storage
    bf, be, bv = (BARS_SPLIT if storage == "split" and emb[-1] > 128 else BARS)[prec]
    assert np.isfinite(f).all()
    assert df <= bf * rms
    assert de <= be * abs(r["energy"])
    assert dv <= bv * vs


def test_wide_rejected_in_fp64():
    """FP64 kernels hold widths up to 128; a wide net asks for mixed precision."""
    from paper_2005_00223_amd.model import DPModel
    spec = _model("cu3", 4.5, (64, 128, 256))
    with pytest.raises(Exception) as ei:
        DPModel(synth.pack_blob(spec), "fp64")
    say(f"[wide] fp64 refusal: {ei.value}")
    assert "mixed" in str(ei.value)


def test_wide_sweep_workload_atom_energies():
    """Largest net of the study on the full sweep workload: per-atom energies
    of 8 sampled atoms against the oracle's per-centre evaluation."""
    from oracle import oracle as O
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload("cu13500")
    spec = synth.copper_model(1, emb=(512, 1024, 2048))
    n = len(w["types"])
    m = DPModel(synth.pack_blob(spec), "fp16")
    say(f"[wide] sweep workload {n} atoms, emb 512-1024-2048")
    e, f, v = m.compute(w["coords"], w["types"], w["box"], keep_intermediates=True)
    ae = m.intermediates(n, spec.M1, spec.M2, spec.nnei, which=("atom_e",))["atom_e"].cpu().numpy()
    assert abs(ae.sum() - float(e)) <= 1e-9 * max(1.0, abs(float(e)))
    idx = np.random.default_rng(5).choice(n, 8, replace=False)
    r = O.Oracle(synth.pack_blob(_quantised(spec, "fp16"))).eval(w["coords"], w["types"], w["box"], centres=idx)
    ref = r["atom_e"]  # in the order of the centres
    d = np.abs(ae[idx] - ref)
    say(f"  sampled |dE_i| max {d.max():.3e} (|E_i| ~ {np.abs(ref).mean():.3e})")
    assert np.isfinite(f.cpu().numpy()).all()
    assert (d <= 2e-3 * np.maximum(1.0, np.abs(ref))).all()


def test_wide_net_deriv_and_atom_energies():
    """dE/dR of every real slot (the per-pair contraction of the backward
    kernel, before the FP64 force pass) and the per-atom energies."""
    from oracle import oracle as O
    from paper_2005_00223_amd.model import DPModel
    x, t, box = _system("cu3")
    spec = _model("cu3", 4.5, (64, 128, 256))
    n = len(t)
    say("[wide] net_deriv cu3 64-128-256 fp16")
    m = DPModel(synth.pack_blob(spec), "fp16")
    m.compute(x, t, box, keep_intermediates=True)
    g = {k: v.cpu().numpy() for k, v in m.intermediates(n, spec.M1, spec.M2, spec.nnei,
                                                        which=("atom_e", "net_deriv")).items()}
    r = O.Oracle(synth.pack_blob(_quantised(spec, "fp16"))).eval(x, t, box, intermediates=True)
    real = r["nlist"] >= 0
    nd, rd = g["net_deriv"][real], r["net_deriv"][real]
    rel = float(np.linalg.norm(nd - rd) / np.linalg.norm(rd))
    de = np.abs(g["atom_e"] - r["atom_e"])
    say(f"  dE/dR relative error {rel:.2e}, max |dE_i| {de.max():.2e}")
    assert rel <= 5e-3
    assert (de <= 1e-4 * np.maximum(1.0, np.abs(r["atom_e"]))).all()


def test_wide_md_matches_oracle_verlet():
    """20 NVE steps of water (two types, four wide nets) against the oracle's
    velocity Verlet on the pre-rounded model."""
    from oracle import oracle as O
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload("water192")
    spec = _model("water192", 6.0, (64, 128, 256))
    t = w["types"]
    v0 = synth.maxwell_boltzmann(w["masses"][t], 300.0, w["vseed"])
    say("[wide] md water192 64-128-256 fp16, 20 steps")
    m = DPModel(synth.pack_blob(spec), "fp16")
    x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda")
    v = torch.tensor(v0, dtype=torch.float64, device="cuda")
    th = m.md_run(x, v, t, w["box"], w["masses"], 0.5, 20, skin=0.2, thermo_every=5)
    assert m.stats()["wide_evals"] >= 20
    ox, ov, oth = O.Oracle(synth.pack_blob(_quantised(spec, "fp16"))).verlet(
        w["coords"], v0, t, w["box"], w["masses"], 0.5, 20, every=5)
    d = x.cpu().numpy() - ox
    d -= w["box"] * np.round(d / w["box"])
    th = th.cpu().numpy()
    say(f"  max |dx| {np.abs(d).max():.2e} A, PE {th[-1, 2]:.6e} vs {oth[-1, 2]:.6e}")
    assert np.abs(d).max() < 1e-5
    assert np.abs(th[:, 2] - oth[:, 2]).max() <= 1e-4 * np.abs(oth[:, 2]).max()


def test_wide_empty_system():
    from paper_2005_00223_amd.model import DPModel
    spec = _model("cu3", 4.5, (64, 128, 256))
    m = DPModel(synth.pack_blob(spec), "fp16")
    e, f, v = m.compute(np.zeros((0, 3)), np.zeros(0, dtype=np.int32), np.full(3, 10.9))
    assert e.item() == 0.0 and f.shape == (0, 3)
    assert np.all(v.cpu().numpy() == 0.0)


@pytest.mark.parametrize("storage", ["split", "mix16"])
def test_wide_sweep_workload_sampled_forces(storage):
    """128-256-512 (both GEMM tile shapes) on the full sweep workload.  dE/dR
    of every real slot of 4 sampled atoms (what the GEMM path computes per
    pair; the oracle evaluates each atom as its only centre), and the total
    force on 2 sampled atoms (the oracle takes the atom and its neighbours as
    centres, which gives that force exactly).  Split storage: dE/dR within
    1e-4 relative and forces within 1e-3 eV/A.  MIX-16 storage: dE/dR within
    10u; forces of this nearly perfect lattice (0.05 A jitter) are small
    differences of large pair terms, so with dE/dR at ~2u the force RMSE is
    3.5% of RMS|F| (0.7% at 0.25 A jitter), per atom up to ~9% (2,916-atom
    run): the per-atom bar is 15% of RMS|F|."""
    from oracle import oracle as O
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload("cu13500")
    spec = synth.copper_model(1, emb=(128, 256, 512))
    x, t, box = w["coords"], w["types"], w["box"]
    n = len(t)
    say(f"[wide] sweep workload {n} atoms, emb 128-256-512, {storage}, sampled dE/dR and forces")
    m = DPModel(synth.pack_blob(spec), "fp16")
    m.set_wide_storage(0 if storage == "split" else 1)
    e, f, v = m.compute(x, t, box, keep_intermediates=True)
    assert m.stats()["wide_evals"] >= 1
    nd = m.intermediates(n, spec.M1, spec.M2, spec.nnei, which=("net_deriv",))["net_deriv"].cpu().numpy()
    f = f.cpu().numpy()
    rms = float(np.sqrt((f ** 2).sum(1).mean()))
    o = O.Oracle(synth.pack_blob(_quantised(spec, "fp16")))
    rng = np.random.default_rng(9)
    for k in rng.choice(n, size=4, replace=False):
        r = o.eval(x, t, box, centres=np.array([k]), intermediates=True)
        real = r["nlist"][0] >= 0
        rd = r["net_deriv"][0][real]
        rel = float(np.linalg.norm(nd[k][real] - rd) / np.linalg.norm(rd))
        say(f"  atom {k}: dE/dR relative error {rel:.2e} over {int(real.sum())} slots")
        assert rel <= (1e-4 if storage == "split" else 5e-3)
    nl, _, _ = o.nlist(x, t, box)
    for k in rng.choice(n, size=2, replace=False):
        cen = np.unique(np.concatenate([[k], nl[k][nl[k] >= 0]]))
        fk = o.eval(x, t, box, centres=cen)["force"][k]
        d = float(np.linalg.norm(f[k] - fk))
        say(f"  atom {k}: |dF| {d:.3e} (|F| {np.linalg.norm(fk):.3e}, RMS|F| {rms:.3e})")
        assert d <= (1e-3 if storage == "split" else 0.15 * rms)
