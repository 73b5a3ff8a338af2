"""Cell-ordered force scatter of the mixed-precision student backward.

Both scatters sum the same FP64 pair forces; only the order of the sums
differs (LDS accumulation per cell plus a 27-part gather, against global
atomics), so forces, energy and virial agree to rounding.  Cases: the
smallest grid the path takes (3 cells per axis, periodic neighbours wrap
onto each other's opposite faces), BF16, the MD driver's skin list, and
cells holding more atoms than the LDS keeps (those atoms fall back to
global atomics).  The oracle case checks the cell path against the FP64
oracle on the model with 16-bit weights, as the mixed student test does
for the atomic path."""
import sys

import numpy as np
import pytest

from paper_2005_00223_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CELL_CAP = 128  # atoms per cell kept in LDS by the kernel


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cell_counts(w, rlist):
    """Atoms per cell of the list grid (side >= rlist), from the coordinates."""
    L = np.asarray(w["box"], dtype=np.float64)
    L = L if L.size == 3 else L.reshape(3, 3).diagonal()
    nc = np.maximum(1, np.floor(L / rlist).astype(int))
    x = np.mod(np.asarray(w["coords"], dtype=np.float64), L)
    c = np.minimum((x / (L / nc)).astype(int), nc - 1)
    idx = (c[:, 0] * nc[1] + c[:, 1]) * nc[2] + c[:, 2]
    return nc, np.bincount(idx, minlength=int(np.prod(nc)))


def _student(spec, seed=12):
    P = synth.random_student_params(spec, seed).astype(np.float64)
    return synth.pack_blob(synth.student_spec(spec, P))


def _run(w, sblob, prec, mode, skin):
    from paper_2005_00223_amd.model import DPModel
    m = DPModel(synth.pack_blob(w["spec"]), prec)
    m.student_set_model(sblob)
    m.student_use(True)
    m.student_judge(0, 1.0)  # no judge: the untrained student's forces themselves are compared
    m.set_force_scatter(mode)
    if skin is None:
        e, f, v = m.compute(w["coords"], w["types"], w["box"])
        out = (float(e), f.cpu().numpy(), np.asarray(v.cpu().numpy()).reshape(-1))
    else:
        x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda")
        vel = torch.zeros_like(x)
        t = torch.tensor(w["types"], dtype=torch.int32, device="cuda")
        F = torch.zeros_like(x)
        th = m.md_run(x, vel, t, w["box"], w["masses"], w["dt_fs"], 0, skin=skin, thermo_every=1, forces=F)
        out = (float(th[0, 2]), F.cpu().numpy(), th[0].cpu().numpy())
    return out, m.stats()["cell_scatter"]


@pytest.mark.parametrize("name,prec,skin", [("cu_cells7", "fp16", None), ("cu_cells10", "bf16", None),
                                            ("cu_cells9", "fp16", 2.0), ("cu_cells10", "fp16", 4.0)])
def test_cell_scatter_matches_atomics(name, prec, skin):
    w = synth.workload(name)
    spec = w["spec"]
    rlist = spec.rcut + (skin or 0.0)
    nc, counts = _cell_counts(w, rlist)
    say(f"[cells] {name} {prec} skin {skin}: grid {tuple(nc)}, atoms per cell {counts.min()}..{counts.max()}")
    assert (nc >= 3).all()
    if skin == 4.0:
        assert counts.max() > CELL_CAP  # the case covers the atomic fallback of full cells
    sblob = _student(spec)
    (e0, f0, v0), n0 = _run(w, sblob, prec, 0, skin)
    (e1, f1, v1), n1 = _run(w, sblob, prec, 1, skin)
    assert n0 >= 1 and n1 == 0
    df = float(np.abs(f0 - f1).max())
    fmax = float(np.abs(f1).max())
    dv = float(np.abs(v0 - v1).max())
    say(f"  max |dF| {df:.3e} (max |F| {fmax:.3f}), |dE| {abs(e0 - e1):.3e}, max |d virial/thermo| {dv:.3e}")
    assert np.isfinite(f0).all()
    assert df <= 1e-10 * max(1.0, fmax)
    assert abs(e0 - e1) <= 1e-9 * max(1.0, abs(e1))
    assert dv <= 1e-9 * max(1.0, float(np.abs(v1).max()))


def test_cell_scatter_matches_oracle():
    """Cell path (3 cells per axis) against the FP64 oracle on the student
    model with its 16-bit weights rounded beforehand."""
    from oracle import oracle as O
    from oracle import student as S
    w = synth.workload("cu_cells7")
    spec = w["spec"]
    P = synth.random_student_params(spec, 12).astype(np.float64)
    sblob = synth.pack_blob(synth.student_spec(spec, P))
    npar = synth.student_np(spec.M1)
    o_w2, o_b2, o_w3, o_b3 = 32, 32 + 512, 32 + 512 + 32, npar - spec.M1
    Pq = P.copy()
    Pq[:, o_w2:o_b2] = S.round16(P[:, o_w2:o_b2], 0)
    Pq[:, o_w3:o_b3] = S.round16(P[:, o_w3:o_b3], 0)
    sq = synth.student_spec(spec, Pq)
    for t in range(spec.ntypes):
        for l in range(2):
            sq.fit_W[t][l] = S.round16(sq.fit_W[t][l], 0)
    say("[cells] oracle cu_cells7 fp16")
    r = O.Oracle(synth.pack_blob(sq)).eval(w["coords"], w["types"], w["box"])
    (e, f, v), ncs = _run(w, sblob, "fp16", 0, None)
    assert ncs >= 1
    rmse = float(np.sqrt(((f - r["force"]) ** 2).sum(1).mean()))
    rms = float(np.sqrt((r["force"] ** 2).sum(1).mean()))
    say(f"  force RMSE {rmse:.3e} (RMS|F| {rms:.3f}), dE/atom {abs(e - r['energy']) / len(w['types']):.3e}")
    assert rmse <= 1e-4 * max(1.0, rms)
    # E_i come out of FP32 fitting layers fed with ~22-bit split activations:
    # relative, not per-atom, agreement (this random model has ~73 eV/atom)
    assert abs(e - r["energy"]) <= 5e-5 * abs(r["energy"])
    vo = np.asarray(r["virial"]).reshape(-1)
    assert np.abs(v - vo).max() <= 1e-4 * max(1.0, float(np.abs(vo).max()))


@pytest.mark.parametrize("name,prec,skin", [("cu_cells7", "fp16", None), ("cu_cells9", "bf16", 2.0),
                                            ("water192", "fp16", None)])
def test_student_table_matches_layers(name, prec, skin):
    """Tabulated second layer (cubic Hermite on 81 points) against the
    evaluated layers, same student and kernels.  The table holds FP64 values
    of h2 and ds*dh2/ds; the interpolant's error is ~ds^4 max|h2^(4)|/384 for
    h2 and ~ds^3 max|h2^(4)|/24 for dh2/ds.  With ds = 1.25 s_max / 80 and
    |W1| up to ~12 (h2^(4) ~ W1^4) the derivative, which the forces carry,
    is good to ~2e-4 of its size per feature; summed over neighbours the
    force error stays below 1e-4 of the RMS force (energies, from h2 itself,
    agree to ~1e-8).  Water's four nets do not fit the LDS with their
    tables, so there the layers are evaluated (asserted)."""
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload(name)
    spec = w["spec"]
    sblob = _student(spec)

    def run(tab):
        m = DPModel(synth.pack_blob(spec), prec)
        m.student_set_model(sblob)
        m.student_use(True)
        m.student_judge(0, 1.0)  # no judge: the untrained student's forces themselves are compared
        m.student_table(tab)
        if skin is None:
            e, f, v = m.compute(w["coords"], w["types"], w["box"])
            used.append(m.stats()["table_evals"])
            return float(e), f.cpu().numpy(), np.asarray(v.cpu().numpy()).reshape(-1)
        x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda")
        t = torch.tensor(w["types"], dtype=torch.int32, device="cuda")
        F = torch.zeros_like(x)
        th = m.md_run(x, torch.zeros_like(x), t, w["box"], w["masses"], w["dt_fs"], 0, skin=skin, thermo_every=1,
                      forces=F)
        used.append(m.stats()["table_evals"])
        return float(th[0, 2]), F.cpu().numpy(), th[0].cpu().numpy()

    say(f"[table] {name} {prec} skin {skin}")
    used = []
    e1, f1, v1 = run(True)
    e0, f0, v0 = run(False)
    assert used[1] == 0
    assert used[0] == (0 if spec.ntypes > 1 else 1)
    n = len(w["types"])
    df = float(np.sqrt(((f1 - f0) ** 2).sum(1).mean()))
    rms = float(np.sqrt((f0 ** 2).sum(1).mean()))
    say(f"  force RMSE table vs layers {df:.3e} (RMS|F| {rms:.3f}), dE/atom {abs(e1 - e0) / n:.3e}")
    assert np.isfinite(f1).all()
    # BF16: the evaluated layers themselves carry ~1e-4 (8-bit weight mantissa,
    # 16-bit split activations), the table does not add to that
    assert df <= (1e-4 if prec == "fp16" else 3e-4) * max(1.0, rms)
    assert abs(e1 - e0) <= 1e-6 * max(1.0, abs(e0))


@pytest.mark.parametrize("mode", [0, 1])
def test_table_defers_nets_beyond_its_range(mode):
    """The table is built over the s range of the first frame it meets; a
    later frame with a neighbour closer than that range allows sends the
    nets of the atoms concerned to the deferred layer pass of the backward
    (both force scatters).  Frame B pushes atom 0 to 0.7 of the smallest
    pair distance of frame A (s = 1/r there, 1.43 x the largest s of A,
    beyond the table's 1.25 x); its forces must match the layers' to the
    table test's bar, which a cubic extrapolated that far would miss."""
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload("cu_cells7")
    spec = w["spec"]
    sblob = _student(spec)
    xa = np.asarray(w["coords"], dtype=np.float64)
    L = np.asarray(w["box"], dtype=np.float64)
    L = L if L.size == 3 else L.reshape(3, 3).diagonal()
    d = xa[None, :, :] - xa[:, None, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    rmin = float(r.min())
    j = int(np.argmin(r[0]))
    xb = xa.copy()
    u = d[0, j] / r[0, j]
    xb[0] = xa[j] - u * 0.7 * rmin  # atom 0 at 0.7 rmin from its nearest neighbour, same direction
    # s = 1/r at the new distance (inside the switch's start) against at most
    # 1/rmin anywhere in frame A: 1/0.7 = 1.43 x the table's reference
    assert 0.7 * rmin < spec.rcut_smth

    def model(tab):
        m = DPModel(synth.pack_blob(spec), "fp16")
        m.student_set_model(sblob)
        m.student_use(True)
        m.student_judge(0, 1.0)  # no judge: the untrained student's forces themselves are compared
        m.student_table(tab)
        m.set_force_scatter(mode)
        return m

    say(f"[table] deferred nets, scatter mode {mode}, rmin {rmin:.3f} A")
    mt = model(True)
    mt.compute(xa, w["types"], w["box"])  # builds the table over frame A's range
    e1, f1, v1 = mt.compute(xb, w["types"], w["box"])
    assert mt.stats()["table_evals"] == 2
    m0 = model(False)
    e0, f0, v0 = m0.compute(xb, w["types"], w["box"])
    f1, f0 = f1.cpu().numpy(), f0.cpu().numpy()
    v1 = np.asarray(v1.cpu().numpy()).reshape(-1)
    v0 = np.asarray(v0.cpu().numpy()).reshape(-1)
    df = float(np.sqrt(((f1 - f0) ** 2).sum(1).mean()))
    rms = float(np.sqrt((f0 ** 2).sum(1).mean()))
    d0 = float(np.abs(f1[0] - f0[0]).max())
    say(f"  force RMSE table vs layers {df:.3e} (RMS|F| {rms:.3f}), atom 0 max |dF| {d0:.3e}, |F_0| "
        f"{np.abs(f0[0]).max():.3f}")
    assert np.isfinite(f1).all()
    assert df <= 1e-4 * max(1.0, rms)
    assert d0 <= 1e-4 * max(1.0, float(np.abs(f0[0]).max()))
    assert np.abs(v1 - v0).max() <= 1e-4 * max(1.0, float(np.abs(v0).max()))
