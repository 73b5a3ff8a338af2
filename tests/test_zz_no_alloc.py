"""dp_compute_noalloc (the entry point that allocates nothing: its workspace
is a static device array) against dp_compute, through the C ABI.

Bar (the FP64 parity bar; both entry points run the same kernels on the same
inputs, so only the order of FP64 force atomics may differ): energy within
1e-10 relative, forces within 1e-9 eV/A, virial within 1e-10 relative to its
largest element.  Each case makes two no-allocation calls in a row, the
second on a smaller system, so the second reuses the first's layout of the
static array."""
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


def _box9(box):
    b = np.asarray(box, dtype=np.float64)
    return [b[0], 0, 0, 0, b[1], 0, 0, 0, b[2]] if b.size == 3 else list(b.reshape(9))


def _ctx(blob, prec):
    from paper_2005_00223_amd import _lib as L
    ctx = L.dp_create(0, torch.cuda.current_stream().cuda_stream)
    L.dp_set_model(ctx, blob, L.PRECISION[prec])
    return ctx


def _run(entry, ctx, w):
    """One evaluation through `entry` (dp_compute or dp_compute_noalloc)
    with caller-owned output tensors; returns host (E, F, V)."""
    n = len(w["types"])
    x = torch.tensor(w["coords"], dtype=torch.float64, device="cuda")
    t = torch.tensor(w["types"], dtype=torch.int32, device="cuda")
    e = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    f = torch.full((n, 3), np.nan, dtype=torch.float64, device="cuda")
    v = torch.full((9,), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    entry(ctx, n, x.data_ptr(), t.data_ptr(), _box9(w["box"]), e.data_ptr(), f.data_ptr(), v.data_ptr())
    torch.cuda.synchronize()
    return e.item(), f.cpu().numpy(), v.cpu().numpy()


def _same(a, b, tag):
    (ea, fa, va), (eb, fb, vb) = a, b
    de = abs(ea - eb) / abs(eb)
    df = float(np.abs(fa - fb).max()) if fb.size else 0.0
    dv = float(np.abs(va - vb).max() / max(np.abs(vb).max(), 1e-300))
    say(f"  {tag}: E rel {de:.2e}, F max {df:.2e} eV/A, virial rel {dv:.2e}")
    assert de <= 1e-10 and df <= 1e-9 and dv <= 1e-10


# (precision, first system, second smaller system): copper in FP64 at up to
# 2,916 atoms (9^3 cells; FP64 copper fits about 3,200), water in FP16 at
# 12,288 atoms, then the 192-atom water box
CASES = [("fp64", "cu_cells9", "cu_cells5"), ("fp16", "water12288", "water192")]


@pytest.mark.parametrize("prec,big,small", CASES)
def test_noalloc_matches_compute(prec, big, small):
    from paper_2005_00223_amd import _lib as L
    wb, ws = synth.workload(big), synth.workload(small)
    blob = synth.pack_blob(wb["spec"])
    say(f"[noalloc] {prec}: {big} ({len(wb['types'])} atoms) then {small} ({len(ws['types'])} atoms)")
    ref_ctx, na_ctx = _ctx(blob, prec), _ctx(blob, prec)
    try:
        ref_b = _run(L.dp_compute, ref_ctx, wb)
        ref_s = _run(L.dp_compute, ref_ctx, ws)
        _same(_run(L.dp_compute_noalloc, na_ctx, wb), ref_b, f"{big} (first call)")
        _same(_run(L.dp_compute_noalloc, na_ctx, ws), ref_s, f"{small} (second call, smaller)")
    finally:
        L.dp_destroy(ref_ctx)
        L.dp_destroy(na_ctx)


def test_noalloc_keeps_context_state_and_rejects_oversize():
    """A context's own lists survive a no-allocation call; a system whose
    workspace exceeds the static array is refused before any launch."""
    from paper_2005_00223_amd import _lib as L
    w = synth.workload("water192")
    blob = synth.pack_blob(w["spec"])
    n, nnei = len(w["types"]), w["spec"].nnei
    say("[noalloc] context state and the size limit")
    ctx = _ctx(blob, "fp64")
    try:
        _run(L.dp_compute, ctx, w)
        nl0 = torch.empty((n, nnei), dtype=torch.int32, device="cuda")
        L.dp_get_nlist(ctx, nl0.data_ptr(), None)
        small = dict(w)
        keep = np.arange(n) < 150
        small.update(coords=w["coords"][keep], types=w["types"][keep])
        _run(L.dp_compute_noalloc, ctx, small)
        nl1 = torch.empty((n, nnei), dtype=torch.int32, device="cuda")
        L.dp_get_nlist(ctx, nl1.data_ptr(), None)
        torch.cuda.synchronize()
        assert torch.equal(nl0, nl1)
        # 12,288 water atoms need about 0.7 GB of FP64 workspace: refused
        big = synth.workload("water12288")
        with pytest.raises(L.DPError) as ei:
            _run(L.dp_compute_noalloc, ctx, big)
        assert ei.value.code == L.DP_E_CAP and "static scratch" in str(ei.value)
        # the context still evaluates normally afterwards
        _same(_run(L.dp_compute_noalloc, ctx, w), _run(L.dp_compute, ctx, w), "water192 after the refusal")
    finally:
        L.dp_destroy(ctx)
