"""DP_MIX_FP32 (the paper's MIX-32 scheme): both networks in FP32 (weights,
environment matrix, matrix-core products, tanh, descriptor, backward),
geometry, the force Jacobian and every sum in FP64, against the FP64
oracle.

Bars: the kernels' arithmetic against the oracle on the weights the kernels
hold (every weight and bias rounded to FP32 beforehand).  What is left is
FP32 rounding (unit u = 2^-24) of the environment matrix and of every
product and sum; the longest reductions are the 1,600-term first fitting
layer and the ~180-neighbour sums of T, for which random rounding gives
about sqrt(K) u = 2^-18.6 relative and the worst case K u = 2^-13.4.  The
bar, 2^-16, sits 6x above the first and 6x below the second: forces
relative to RMS|F|, the virial relative to its largest element, the energy
relative to itself.  Measured (cu 500 / water 192 / cu 32,000): forces
1.0e-5 / 7.8e-7 / 1.2e-5, energy 9.4e-8 / 1.2e-8 / 1.7e-8, virial 2.2e-8 /
1.3e-8 / 2.1e-8.  The neighbour list is the FP64 one, bit for bit."""
import copy
import sys

import numpy as np
import pytest

from paper_2005_00223_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BAR = 2.0 ** -16


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle(blob):
    from oracle import oracle as O
    return O.Oracle(blob)


def _round32(spec):
    """The spec with every weight and bias rounded to FP32 (kept in FP64)."""
    q = copy.deepcopy(spec)
    r = lambda a: np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
    for t in range(spec.ntypes):
        for u in range(spec.ntypes):
            for l in range(len(spec.emb)):
                q.emb_W[t][u][l] = r(spec.emb_W[t][u][l])
                q.emb_b[t][u][l] = r(spec.emb_b[t][u][l])
        for l in range(len(spec.fit_W[t])):
            q.fit_W[t][l] = r(spec.fit_W[t][l])
            q.fit_b[t][l] = r(spec.fit_b[t][l])
    return q


def _frmse(a, b):
    return float(np.sqrt(((a - b) ** 2).sum(1).mean()))


@pytest.mark.parametrize("name", ["cu_cells5", "water192", "cu32000"])
def test_fp32_matches_oracle(name):
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload(name)
    blob = synth.pack_blob(w["spec"])
    n = len(w["types"])
    say(f"[fp32] {name}: {n} atoms")
    m = DPModel(blob, "fp32")
    e, f, v = m.compute(w["coords"], w["types"], w["box"])
    e, f, v = e.item(), f.cpu().numpy(), v.cpu().numpy()
    q = _oracle(synth.pack_blob(_round32(w["spec"]))).eval(w["coords"], w["types"], w["box"])
    r = _oracle(blob).eval(w["coords"], w["types"], w["box"])
    rms = np.sqrt((q["force"] ** 2).sum(1).mean())
    kf = _frmse(f, q["force"]) / rms
    ke = abs(e - q["energy"]) / abs(q["energy"])
    kv = np.abs(v - q["virial"]).max() / np.abs(q["virial"]).max()
    rmse = _frmse(f, r["force"])
    say(f"  kernel arithmetic (vs FP32-rounded-weight oracle): force {kf:.2e} x RMS|F|, energy {ke:.2e} rel, "
        f"virial {kv:.2e} rel; vs the model: force RMSE {rmse:.3e} eV/A (RMS|F| {rms:.3f}), "
        f"energy error per atom {abs(e - r['energy']) / n:.3e} eV")
    assert kf <= BAR and ke <= BAR and kv <= BAR
    nl, _ = m.nlist(n, w["spec"].nnei, w["spec"].ntypes)
    onl, _, _ = _oracle(blob).nlist(w["coords"], w["types"], w["box"])
    np.testing.assert_array_equal(nl.cpu().numpy(), onl)


def test_precision_switches_keep_fp32_results():
    """FP64 -> FP32 -> FP16 -> FP32 on one context: both FP32 evaluations
    agree bit for bit (the FP32 weights and buffers do not depend on what
    ran before) and lie within the bar of the FP64 one."""
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload("cu_cells5")
    blob = synth.pack_blob(w["spec"])
    m = DPModel(blob, "fp64")
    e64, f64, _ = m.compute(w["coords"], w["types"], w["box"])
    m.set_precision("fp32")
    e1, f1, v1 = m.compute(w["coords"], w["types"], w["box"])
    f1 = f1.cpu().numpy().copy()
    m.set_precision("fp16")
    m.compute(w["coords"], w["types"], w["box"])
    m.set_precision("fp32")
    e2, f2, v2 = m.compute(w["coords"], w["types"], w["box"])
    f2 = f2.cpu().numpy()
    say(f"[fp32] switches: E {e1.item():.12f} / {e2.item():.12f}, FP64 {e64.item():.12f}")
    f64 = f64.cpu().numpy()
    rms = np.sqrt((f64 ** 2).sum(1).mean())
    assert abs(e1.item() - e64.item()) <= BAR * abs(e64.item())
    assert _frmse(f1, f64) <= BAR * rms
    # the force sums are FP64 atomics, whose order may differ between runs
    assert abs(e1.item() - e2.item()) <= 1e-12 * abs(e64.item())
    np.testing.assert_allclose(f2, f1, rtol=0, atol=1e-12 * rms)


def test_fp32_md_and_adjoint_match_fp64():
    """MIX-32 through the other entry points: 20 velocity-Verlet steps
    (dp_md_run) against the FP64 run from the same start (positions within
    1e-6 A, thermo columns within the bar) and the forward / adjoint pair
    (dp_energy, dp_energy_backward) against dp_compute in FP32 (the same
    kernels: energy and forces equal to 1e-12)."""
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload("water192")
    blob = synth.pack_blob(w["spec"])
    t = w["types"]
    v0 = synth.maxwell_boltzmann(w["masses"][t], 300.0, w["vseed"])
    out = {}
    for prec in ("fp64", "fp32"):
        m = DPModel(blob, prec)
        x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda")
        v = torch.tensor(v0, dtype=torch.float64, device="cuda")
        th = m.md_run(x, v, t, w["box"], w["masses"], 0.5, 20, skin=0.2, thermo_every=5)
        out[prec] = (x.cpu().numpy(), th.cpu().numpy(), m)
    d = out["fp32"][0] - out["fp64"][0]
    d -= w["box"] * np.round(d / w["box"])
    th32, th64 = out["fp32"][1], out["fp64"][1]
    scale = np.abs(th64[:, 1:4]).max()
    say(f"[fp32] md: max |dx| {np.abs(d).max():.2e} A, thermo (KE, PE, E) {np.abs(th32[:, 1:4] - th64[:, 1:4]).max() / scale:.2e} "
        f"of their largest")
    assert np.abs(d).max() < 1e-6
    assert np.abs(th32[:, 1:4] - th64[:, 1:4]).max() <= BAR * scale
    m = out["fp32"][2]
    e, f, _ = m.compute(w["coords"], t, w["box"])
    ea = m.energy(w["coords"], t, w["box"])
    fa, _ = m.energy_backward(1.0)
    rms = float(np.sqrt((f.cpu().numpy() ** 2).sum(1).mean()))
    assert abs(ea.item() - e.item()) <= 1e-12 * abs(e.item())
    np.testing.assert_allclose(fa.cpu().numpy(), f.cpu().numpy(), rtol=0, atol=1e-12 * rms)
