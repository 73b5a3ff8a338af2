"""torch-facing wrapper of the C ABI: tensors for device memory, the current
HIP stream for ordering.  All arithmetic happens in libdpmi's kernels."""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


def _box9(box) -> list:
    b = np.asarray(box, dtype=np.float64)
    if b.size == 3:
        return [b[0], 0, 0, 0, b[1], 0, 0, 0, b[2]]
    return list(b.reshape(9))


def _ptr(t):
    return None if t is None else t.data_ptr()


class DPModel:
    """A loaded Deep Potential model on one GPU.

    blob: bytes in the DPMIBLOB layout.  precision: "fp64", "fp32" (the
    paper's MIX-32), "fp16" or "bf16" (the 16-bit mixed-precision kernels)."""

    def __init__(self, blob: bytes, precision: str = "fp64", device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("DPModel needs a ROCm GPU; there is no CPU path")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        stream = torch.cuda.current_stream(self.device)
        self.ctx = L.dp_create(self.device.index, stream.cuda_stream)
        self.precision = precision
        self.eval_id = 0   # bumped by every call that replaces the library's forward state
        L.dp_set_model(self.ctx, bytes(blob), L.PRECISION[precision])

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            L.dp_destroy(ctx)
            self.ctx = None

    def set_precision(self, precision: str):
        self.eval_id += 1
        L.dp_set_precision(self.ctx, L.PRECISION[precision])
        self.precision = precision

    def _dev(self, x, dtype):
        t = torch.as_tensor(x, dtype=dtype)
        return t.to(self.device).contiguous()

    def compute(self, coords, types, box, keep_intermediates=False):
        """Energy (eV, 0-d), forces [N,3] (eV/A), virial [3,3] (eV) as
        double tensors on the GPU."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        f = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty(9, dtype=torch.float64, device=self.device)
        self.eval_id += 1
        L.dp_keep_intermediates(self.ctx, keep_intermediates)
        L.dp_compute(self.ctx, n, _ptr(x), _ptr(t), _box9(box), _ptr(e), _ptr(f), _ptr(v))
        self._n = n
        return e[0], f, v.view(3, 3)

    def compute_local(self, coords, types, box, n_local):
        """Rank-share evaluation: atoms [0, n_local) are centres, the rest
        ghosts (neighbours only).  Energy (0-d), forces [N,3] on every atom
        (ghosts included), virial [3,3]."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        f = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty(9, dtype=torch.float64, device=self.device)
        self.eval_id += 1
        L.dp_compute_local(self.ctx, n_local, n, _ptr(x), _ptr(t), _box9(box), _ptr(e), _ptr(f), _ptr(v))
        return e[0], f, v.view(3, 3)

    def scatter_add_forces(self, index, f_in, f_out):
        """f_out[index[k]] += f_in[k] on the device (reverse communication)."""
        idx = self._dev(index, torch.int32)
        assert f_in.dtype == torch.float64 and f_out.dtype == torch.float64 and f_in.is_contiguous()
        L.dp_scatter_add_forces(self.ctx, idx.shape[0], _ptr(idx), _ptr(f_in), _ptr(f_out))

    def energy(self, coords, types, box):
        """Forward half only (0-d energy tensor); keeps the state for
        energy_backward."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        self.eval_id += 1
        L.dp_energy(self.ctx, x.shape[0], _ptr(x), _ptr(t), _box9(box), _ptr(e))
        self._n = x.shape[0]
        return e[0]

    def energy_backward(self, grad_energy=1.0):
        """Adjoint of the last energy(): (forces = -g dE/dr [N,3], g * virial [3,3])."""
        f = torch.empty((getattr(self, "_n", 0), 3), dtype=torch.float64, device=self.device)
        v = torch.empty(9, dtype=torch.float64, device=self.device)
        L.dp_energy_backward(self.ctx, float(grad_energy), _ptr(f), _ptr(v))
        return f, v.view(3, 3)

    def nlist(self, natoms, nnei, ntypes, with_list=True):
        """(nlist [N, nnei], nreal [N, ntypes]) of the last evaluation;
        with_list=False fetches only the real-neighbour counts."""
        nl = torch.empty((natoms, nnei), dtype=torch.int32, device=self.device) if with_list else None
        nr = torch.empty((natoms, ntypes), dtype=torch.int32, device=self.device)
        L.dp_get_nlist(self.ctx, _ptr(nl), _ptr(nr))
        return nl, nr

    def intermediates(self, natoms, M1, M2, nnei, which=("atom_e", "T", "D", "net_deriv")):
        """Per-atom intermediates of the last evaluation (net_deriv needs
        compute(..., keep_intermediates=True); its padded slots are 0)."""
        out = {}
        if "atom_e" in which:
            out["atom_e"] = torch.empty(natoms, dtype=torch.float64, device=self.device)
        if "T" in which:
            out["T"] = torch.empty((natoms, M1, 4), dtype=torch.float64, device=self.device)
        if "D" in which:
            out["D"] = torch.empty((natoms, M1 * M2), dtype=torch.float64, device=self.device)
        if "net_deriv" in which:
            out["net_deriv"] = torch.empty((natoms, nnei, 4), dtype=torch.float64, device=self.device)
        L.dp_get_intermediates(self.ctx, *(_ptr(out.get(k)) for k in ("atom_e", "T", "D", "net_deriv")))
        return out

    def md_run(self, coords, vel, types, box, masses, dt, nsteps, skin=2.0, thermo_every=20, forces=None):
        """NVE velocity Verlet in place on coords/vel (double CUDA tensors).
        Returns the thermo tensor [nsteps//thermo_every + 1, 6]."""
        assert coords.dtype == torch.float64 and vel.dtype == torch.float64 and coords.is_cuda and vel.is_cuda
        t = self._dev(types, torch.int32)
        n = coords.shape[0]
        rows = nsteps // thermo_every + 1 if thermo_every > 0 else 0
        th = torch.zeros((max(rows, 1), 6), dtype=torch.float64, device=self.device)
        m = list(np.asarray(masses, dtype=np.float64)) + [1.0] * (8 - len(masses))
        self.eval_id += 1
        L.dp_md_run(self.ctx, n, _ptr(coords), _ptr(vel), _ptr(t), _box9(box), m, dt, skin, nsteps,
                    max(thermo_every, 1), _ptr(th) if rows else None, _ptr(forces))
        return th[:rows]

    def stats(self):
        return L.dp_get_stats(self.ctx)

    def student_table(self, on: bool):
        """Tabulated student layers (default on; mixed precision only)."""
        self.eval_id += 1
        L.dp_student_table(self.ctx, on)

    def set_force_scatter(self, mode: int):
        """0: cell-ordered LDS scatter where the path allows it (default);
        1: FP64 global atomics for every pair force."""
        L.dp_set_force_scatter(self.ctx, mode)

    def set_wide_storage(self, mode: int):
        """Wide embedding nets: 0 = activations as hi + lo 16-bit pairs
        (default, accurate); 1 = one 16-bit value each (MIX-16 storage)."""
        self.eval_id += 1
        L.dp_set_wide_storage(self.ctx, mode)

    # ---- student embedding net -------------------------------------------
    @staticmethod
    def student_cfg(**kw) -> "L.dp_student_cfg":
        """The library defaults (batch 4096, 500 Adam steps, lr 1e-3, ...),
        with any field overridden by keyword."""
        cfg = L.dp_student_default_cfg()
        for k, v in kw.items():
            if k not in dict(L.dp_student_cfg._fields_):
                raise KeyError(k)
            setattr(cfg, k, v)
        return cfg

    def student_train(self, **kw) -> float:
        """Fit the student to the teacher on the last evaluated frame; returns
        the held-out relative RMSE of G (or the last Adam loss without refit)."""
        self.eval_id += 1
        return L.dp_student_train(self.ctx, self.student_cfg(**kw))

    def student_use(self, on=True):
        self.eval_id += 1
        L.dp_student_use(self.ctx, on)

    def student_judge(self, every=20, max_force_rmse=1e-3, sample_side=0.0):
        """Judge period and threshold; sample_side > 0 (A) judges the atoms
        of a cube of that side (teacher on the cube and its rc margin)."""
        L.dp_student_judge(self.ctx, every, max_force_rmse)
        L.dp_student_judge_sample(self.ctx, sample_side)

    def student_model(self) -> bytes:
        return L.dp_student_get_model(self.ctx)

    def student_set_model(self, blob: bytes):
        self.eval_id += 1
        L.dp_student_set_model(self.ctx, bytes(blob))

    def _student_np(self, ntypes, M1):
        return ntypes * ntypes, 16 + 16 + 16 * 32 + 32 + 32 * M1 + M1

    def student_params(self, ntypes, M1) -> np.ndarray:
        nets, npar = self._student_np(ntypes, M1)
        out = np.empty((nets, npar), dtype=np.float32)
        L.dp_student_get_params(self.ctx, out.ctypes.data)
        return out

    def student_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        L.dp_student_set_params(self.ctx, p.ctypes.data)

    def student_batch_grad(self, ntypes, M1, seed, step, batch):
        """(s [nets, batch], loss [nets], grad [nets, np]) of one Adam batch at
        the current parameters (no update)."""
        nets, npar = self._student_np(ntypes, M1)
        s = np.empty((nets, batch), dtype=np.float64)
        loss = np.empty(nets, dtype=np.float64)
        g = np.empty((nets, npar), dtype=np.float32)
        L.dp_student_batch_grad(self.ctx, seed, step, batch, s.ctypes.data, loss.ctypes.data, g.ctypes.data)
        return s, loss, g

    def enable_timing(self, on=True):
        L.dp_enable_timing(self.ctx, on)

    def timing(self, name):
        return L.dp_get_timing(self.ctx, name)


class DPEnergy(torch.autograd.Function):
    """E(coords[, strain]) with the library's hand-written adjoint as the
    backward.

    forward runs dp_energy (list, environment matrix, embedding +
    descriptor, fitting net); backward runs dp_energy_backward, the fitting
    and embedding backward with the ProdForce and ProdVirial passes, and
    returns grad_E * dE/dcoords = -grad_E * F and, when a strain tensor is
    given, grad_E * dE/dstrain = -grad_E * virial.  Use as
    ``E = DPEnergy.apply(coords, model, types, box)`` or
    ``E = DPEnergy.apply(coords, model, types, box, strain)``.

    strain: a 3x3 double tensor eps (usually zeros with requires_grad): the
    energy is evaluated at x -> (I + eps) x with the box scaled the same way
    (diagonal eps only, as boxes are orthorhombic; off-diagonal entries must
    be zero, their gradient is still returned).  The virial is
    Xi = -dE/deps at eps = 0 (Sec. V-B, ProdVirial).

    Each forward records the model's evaluation id; if other evaluations ran
    on the model before this backward (two applies in one graph, or a
    compute in between), the backward first re-runs the forward on the
    saved coordinates (with the model's settings at that time), so every
    gradient belongs to its own coordinates."""

    @staticmethod
    def forward(ctx, coords, model, types, box, strain=None):
        x = coords.detach()
        b = np.asarray(_box9(box), dtype=np.float64).reshape(3, 3)
        a = None
        if strain is not None:
            eps = strain.detach().to("cpu", torch.float64).numpy().reshape(3, 3)
            if np.any(eps - np.diag(np.diag(eps))):
                raise ValueError("DPEnergy: only a diagonal strain can be applied (orthorhombic boxes)")
            a = np.eye(3) + eps
            x = x @ torch.as_tensor(a.T, dtype=x.dtype, device=x.device)
            b = b @ a.T
        ctx.model, ctx.types, ctx.box, ctx.a = model, types, b.reshape(9), a
        ctx.x = x
        e = model.energy(x, types, ctx.box)
        ctx.eval_id = model.eval_id
        return e

    @staticmethod
    def backward(ctx, grad_e):
        m = ctx.model
        if m.eval_id != ctx.eval_id:
            m.energy(ctx.x, ctx.types, ctx.box)
            ctx.eval_id = m.eval_id
        # the library works with one host scalar: a CUDA grad is read back
        f, vir = m.energy_backward(float(grad_e))
        gs = None
        if ctx.a is None:
            gx = -f
        else:
            at = torch.as_tensor(ctx.a, dtype=f.dtype, device=f.device)
            gx = -f @ at
            gs = -vir @ torch.linalg.inv(at).T
        return gx, None, None, None, gs
