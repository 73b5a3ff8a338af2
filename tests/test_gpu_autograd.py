"""The hand-written adjoint (dp_energy_backward) behind torch.autograd:
gradients equal -F from the fused evaluation, scale with the upstream
gradient, match central finite differences of the GPU's own per-atom
energies, and match the FP64 oracle's forces."""
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


def _setup(name, prec="fp64"):
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload(name)
    blob = synth.pack_blob(w["spec"])
    return w, blob, DPModel(blob, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_grad_equals_minus_force(prec):
    from paper_2005_00223_amd.model import DPEnergy
    w, blob, m = _setup("water192", prec)
    say(f"[autograd] water192 {prec}")
    x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda", requires_grad=True)
    e = DPEnergy.apply(x, m, w["types"], w["box"])
    (3.0 * e).backward()
    e2, f2, _ = m.compute(w["coords"], w["types"], w["box"])
    assert e.item() == e2.item()
    torch.testing.assert_close(x.grad, -3.0 * f2, rtol=0, atol=1e-12)


def test_backward_requires_forward_state():
    from paper_2005_00223_amd import _lib
    w, blob, m = _setup("water192")
    say("[autograd] state")
    m.compute(w["coords"], w["types"], w["box"])
    with pytest.raises(_lib.DPError):
        m.energy_backward(1.0)


def test_finite_differences_cu32000():
    """Central differences (h = 1e-5 A) of the local energy
    sum_{i in {k} + N(k)} E_i on 64 sampled atoms of the 32,000-atom copper
    system against the autograd gradient."""
    from paper_2005_00223_amd.model import DPEnergy
    w, blob, m = _setup("cu32000")
    spec = w["spec"]
    n = len(w["types"])
    say("[autograd] cu32000 finite differences")
    x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda", requires_grad=True)
    e = DPEnergy.apply(x, m, w["types"], w["box"])
    e.backward()
    grad = x.grad.cpu().numpy()
    m.compute(w["coords"], w["types"], w["box"])
    nl, _ = m.nlist(n, spec.nnei, spec.ntypes)
    nl = nl.cpu().numpy()
    rng = np.random.default_rng(64)
    h = 1e-5
    worst = 0.0
    for k in rng.choice(n, size=64, replace=False):
        cen = np.unique(np.concatenate([[k], nl[k][nl[k] >= 0]]))
        for a in range(3):
            el = []
            for sgn in (1.0, -1.0):
                xs = w["coords"].copy()
                xs[k, a] += sgn * h
                m.compute(xs, w["types"], w["box"])
                ae = m.intermediates(n, spec.M1, spec.M2, spec.nnei, which=("atom_e",))["atom_e"]
                el.append(ae[torch.as_tensor(cen, device="cuda")].sum().item())
            fd = (el[0] - el[1]) / (2 * h)
            worst = max(worst, abs(fd - grad[k, a]))
    say(f"  max |FD - grad| = {worst:.2e} eV/A")
    assert worst < 1e-6


def test_grad_matches_oracle_forces():
    from oracle import oracle as O
    from paper_2005_00223_amd.model import DPEnergy
    w, blob, m = _setup("cu_cells5")
    say("[autograd] vs oracle")
    x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda", requires_grad=True)
    DPEnergy.apply(x, m, w["types"], w["box"]).backward()
    r = O.Oracle(blob).eval(w["coords"], w["types"], w["box"])
    assert np.abs(x.grad.cpu().numpy() + r["force"]).max() < 1e-9


def test_two_applies_one_backward():
    """Two forwards on one model before a single backward: each input gets
    the gradient of its own coordinates (the backward re-runs a forward
    that a later evaluation replaced)."""
    from paper_2005_00223_amd.model import DPEnergy
    w, blob, m = _setup("water192")
    say("[autograd] two applies, one backward")
    x0 = w["coords"]
    x1 = x0 + np.random.default_rng(3).normal(scale=0.05, size=x0.shape)
    a = torch.tensor(x0, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(x1, dtype=torch.float64, device="cuda", requires_grad=True)
    e = DPEnergy.apply(a, m, w["types"], w["box"]) + 2.0 * DPEnergy.apply(b, m, w["types"], w["box"])
    e.backward()
    _, fa, _ = m.compute(x0, w["types"], w["box"])
    _, fb, _ = m.compute(x1, w["types"], w["box"])
    assert (fa - fb).abs().max().item() > 1e-3      # the two frames differ
    torch.testing.assert_close(a.grad, -fa, rtol=0, atol=1e-12)
    torch.testing.assert_close(b.grad, -2.0 * fb, rtol=0, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp16", "bf16"])
def test_strain_gradient_is_minus_virial_cu32000(prec):
    """The virial through autograd: dE/d(strain) at zero strain equals -Xi
    of the fused evaluation, and for FP64 a central difference of E under
    a diagonal strain (atoms and box scaled, h = 1e-5) and the oracle's
    virial; for the 16-bit policies the FD and oracle bars are relative to
    the trace."""
    from oracle import oracle as O
    from paper_2005_00223_amd.model import DPEnergy
    w, blob, m = _setup("cu32000", prec)
    say(f"[autograd] cu32000 {prec} strain gradient")
    x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.zeros((3, 3), dtype=torch.float64, device="cuda", requires_grad=True)
    DPEnergy.apply(x, m, w["types"], w["box"], eps).backward()
    _, f, vir = m.compute(w["coords"], w["types"], w["box"])
    torch.testing.assert_close(eps.grad, -vir, rtol=0, atol=1e-12 * vir.abs().max().item())
    torch.testing.assert_close(x.grad, -f, rtol=0, atol=1e-12)
    g = eps.grad.cpu().numpy()
    h = 1e-5
    scale = np.abs(np.diag(g)).max()
    for a in range(3):
        e = []
        for sgn in (1.0, -1.0):
            s = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
            s[a, a] = sgn * h
            e.append(DPEnergy.apply(x.detach(), m, w["types"], w["box"], s).item())
        fd = (e[0] - e[1]) / (2 * h)
        say(f"  dE/deps_{a}{a}: FD {fd:.9e}  autograd {g[a, a]:.9e}")
        if prec == "fp64":
            assert abs(fd - g[a, a]) <= 1e-7 * scale
    if prec == "fp64":
        ref = O.Oracle(blob).eval(w["coords"], w["types"], w["box"])["virial"]
        err = np.abs(-g - ref).max() / np.abs(ref).max()
        say(f"  virial vs oracle: {err:.2e} relative")
        assert err < 1e-10
