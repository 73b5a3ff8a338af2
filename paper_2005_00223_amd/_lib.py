"""ctypes binding of libdpmi.so, one Python function per C entry point of
include/dpmi.h (argument marshalling only; every step runs in the HIP
kernels).  Importing this module loads the library and fails loudly if it is
missing: there is no CPU fallback."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpmi.so")

DP_OK, DP_E_ARG, DP_E_NOMODEL, DP_E_MODEL, DP_E_BOX, DP_E_TYPE, DP_E_OOM, DP_E_HIP, DP_E_NONFINITE, DP_E_CAP = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
DP_FP64, DP_MIX_FP32, DP_MIX_BF16, DP_MIX_FP16 = 0, 1, 2, 3
PRECISION = {"fp64": DP_FP64, "fp32": DP_MIX_FP32, "fp16": DP_MIX_FP16, "bf16": DP_MIX_BF16}

EXPORTS = ("dp_create", "dp_set_model", "dp_set_precision", "dp_compute", "dp_compute_noalloc", "dp_compute_local",
           "dp_scatter_add_forces", "dp_energy", "dp_energy_backward",
           "dp_get_nlist", "dp_keep_intermediates",
           "dp_get_intermediates", "dp_get_stats", "dp_set_force_scatter", "dp_set_wide_storage", "dp_student_table", "dp_md_run", "dp_enable_timing", "dp_get_timing",
           "dp_student_default_cfg", "dp_student_train", "dp_student_get_params", "dp_student_set_params",
           "dp_student_batch_grad", "dp_student_use", "dp_student_judge", "dp_student_judge_sample",
           "dp_student_get_model",
           "dp_student_set_model", "dp_last_error", "dp_destroy")


class dp_stats(C.Structure):
    _fields_ = [("natoms", C.c_int64), ("sel_overflow", C.c_int64), ("max_real", C.c_int32 * 8),
                ("nlist_builds", C.c_int64), ("evaluations", C.c_int64), ("cand_cap", C.c_int64),
                ("student_evals", C.c_int64), ("teacher_fallbacks", C.c_int64), ("last_judge_rmse", C.c_double),
                ("judge_atoms", C.c_int64), ("cell_scatter", C.c_int64), ("table_evals", C.c_int64),
                ("wide_evals", C.c_int64)]


class dp_student_cfg(C.Structure):
    _fields_ = [("batch", C.c_int64), ("adam_steps", C.c_int64), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("ls_samples", C.c_int64), ("ridge", C.c_double),
                ("seed", C.c_uint64), ("init", C.c_int32), ("refit", C.c_int32)]


class DPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dpmi error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libdpmi.so (built by paper_2005_00223_amd.build) and declare
    the prototypes.  Raises ImportError when the library is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2005_00223_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, I64, I32 = C.c_void_p, C.c_int64, C.c_int
    D = C.c_double
    sig = {
        "dp_create": (I32, [C.POINTER(P), I32, P]),
        "dp_set_model": (I32, [P, C.c_char_p, C.c_size_t, I32]),
        "dp_set_precision": (I32, [P, I32]),
        "dp_compute": (I32, [P, I64, P, P, P, P, P, P]),
        "dp_compute_noalloc": (I32, [P, I64, P, P, P, P, P, P]),
        "dp_compute_local": (I32, [P, I64, I64, P, P, P, P, P, P]),
        "dp_scatter_add_forces": (I32, [P, I64, P, P, P]),
        "dp_energy": (I32, [P, I64, P, P, P, P]),
        "dp_energy_backward": (I32, [P, D, P, P]),
        "dp_get_nlist": (I32, [P, P, P]),
        "dp_keep_intermediates": (I32, [P, I32]),
        "dp_get_intermediates": (I32, [P, P, P, P, P]),
        "dp_get_stats": (I32, [P, C.POINTER(dp_stats)]),
        "dp_set_force_scatter": (I32, [P, I32]),
        "dp_set_wide_storage": (I32, [P, I32]),
        "dp_student_table": (I32, [P, I32]),
        "dp_md_run": (I32, [P, I64, P, P, P, P, P, D, D, I64, I64, P, P]),
        "dp_enable_timing": (I32, [P, I32]),
        "dp_get_timing": (I32, [P, C.c_char_p, C.POINTER(D)]),
        "dp_student_default_cfg": (I32, [C.POINTER(dp_student_cfg)]),
        "dp_student_train": (I32, [P, C.POINTER(dp_student_cfg), C.POINTER(D)]),
        "dp_student_get_params": (I32, [P, P]),
        "dp_student_set_params": (I32, [P, P]),
        "dp_student_batch_grad": (I32, [P, C.c_uint64, I64, I64, P, P, P]),
        "dp_student_use": (I32, [P, I32]),
        "dp_student_judge": (I32, [P, I64, D]),
        "dp_student_judge_sample": (I32, [P, D]),
        "dp_student_get_model": (I32, [P, P, C.c_size_t, C.POINTER(C.c_size_t)]),
        "dp_student_set_model": (I32, [P, C.c_char_p, C.c_size_t]),
        "dp_last_error": (C.c_char_p, [P]),
        "dp_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(ctx, rc):
    if rc != DP_OK:
        msg = lib().dp_last_error(ctx)
        raise DPError(rc, msg.decode() if msg else "")
    return rc


# thin wrappers with the C names ------------------------------------------------
def dp_create(device: int, stream_handle: int):
    h = C.c_void_p()
    rc = lib().dp_create(C.byref(h), int(device), C.c_void_p(stream_handle or None))
    if rc != DP_OK:
        raise DPError(rc, "dp_create failed")
    return h


def dp_set_model(ctx, blob: bytes, precision: int):
    return check(ctx, lib().dp_set_model(ctx, blob, len(blob), int(precision)))


def dp_set_precision(ctx, precision: int):
    return check(ctx, lib().dp_set_precision(ctx, int(precision)))


def dp_compute(ctx, natoms, coords_ptr, types_ptr, box9, e_ptr, f_ptr, v_ptr):
    box = (C.c_double * 9)(*[float(b) for b in box9])
    return check(ctx, lib().dp_compute(ctx, int(natoms), coords_ptr, types_ptr, box, e_ptr, f_ptr, v_ptr))


def dp_compute_noalloc(ctx, natoms, coords_ptr, types_ptr, box9, e_ptr, f_ptr, v_ptr):
    box = (C.c_double * 9)(*[float(b) for b in box9])
    return check(ctx, lib().dp_compute_noalloc(ctx, int(natoms), coords_ptr, types_ptr, box, e_ptr, f_ptr, v_ptr))


def dp_compute_local(ctx, n_local, natoms, coords_ptr, types_ptr, box9, e_ptr, f_ptr, v_ptr):
    box = (C.c_double * 9)(*[float(b) for b in box9])
    return check(ctx, lib().dp_compute_local(ctx, int(n_local), int(natoms), coords_ptr, types_ptr, box, e_ptr, f_ptr,
                                             v_ptr))


def dp_scatter_add_forces(ctx, n, index_ptr, f_in_ptr, f_out_ptr):
    return check(ctx, lib().dp_scatter_add_forces(ctx, int(n), index_ptr, f_in_ptr, f_out_ptr))


def dp_energy(ctx, natoms, coords_ptr, types_ptr, box9, e_ptr):
    box = (C.c_double * 9)(*[float(b) for b in box9])
    return check(ctx, lib().dp_energy(ctx, int(natoms), coords_ptr, types_ptr, box, e_ptr))


def dp_energy_backward(ctx, grad_energy, f_ptr, v_ptr):
    return check(ctx, lib().dp_energy_backward(ctx, float(grad_energy), f_ptr, v_ptr))


def dp_get_nlist(ctx, nlist_ptr, nreal_ptr):
    return check(ctx, lib().dp_get_nlist(ctx, nlist_ptr, nreal_ptr))


def dp_keep_intermediates(ctx, keep: bool):
    return check(ctx, lib().dp_keep_intermediates(ctx, int(bool(keep))))


def dp_get_intermediates(ctx, atom_e_ptr, T_ptr, D_ptr, nd_ptr):
    return check(ctx, lib().dp_get_intermediates(ctx, atom_e_ptr, T_ptr, D_ptr, nd_ptr))


def dp_get_stats(ctx) -> dict:
    s = dp_stats()
    check(ctx, lib().dp_get_stats(ctx, C.byref(s)))
    return {k: (list(getattr(s, k)) if k == "max_real" else getattr(s, k)) for k, _ in dp_stats._fields_}


def dp_md_run(ctx, natoms, x_ptr, v_ptr, t_ptr, box9, masses, dt, skin, nsteps, every, thermo_ptr, f_ptr):
    box = (C.c_double * 9)(*[float(b) for b in box9])
    m = (C.c_double * 8)(*[float(v) for v in masses])
    return check(ctx, lib().dp_md_run(ctx, int(natoms), x_ptr, v_ptr, t_ptr, box, m, float(dt), float(skin),
                                      int(nsteps), int(every), thermo_ptr, f_ptr))


def dp_set_force_scatter(ctx, mode: int):
    return check(ctx, lib().dp_set_force_scatter(ctx, int(mode)))


def dp_set_wide_storage(ctx, mode: int):
    return check(ctx, lib().dp_set_wide_storage(ctx, int(mode)))


def dp_student_table(ctx, on: bool):
    return check(ctx, lib().dp_student_table(ctx, int(bool(on))))


def dp_enable_timing(ctx, on: bool):
    return check(ctx, lib().dp_enable_timing(ctx, int(bool(on))))


def dp_get_timing(ctx, name: str) -> float:
    v = C.c_double()
    check(ctx, lib().dp_get_timing(ctx, name.encode(), C.byref(v)))
    return v.value


def dp_student_default_cfg() -> dp_student_cfg:
    cfg = dp_student_cfg()
    lib().dp_student_default_cfg(C.byref(cfg))
    return cfg


def dp_student_train(ctx, cfg: dp_student_cfg) -> float:
    r = C.c_double()
    check(ctx, lib().dp_student_train(ctx, C.byref(cfg), C.byref(r)))
    return r.value


def dp_student_get_params(ctx, out_ptr):
    return check(ctx, lib().dp_student_get_params(ctx, out_ptr))


def dp_student_set_params(ctx, in_ptr):
    return check(ctx, lib().dp_student_set_params(ctx, in_ptr))


def dp_student_batch_grad(ctx, seed, step, batch, s_ptr, loss_ptr, grad_ptr):
    return check(ctx, lib().dp_student_batch_grad(ctx, int(seed), int(step), int(batch), s_ptr, loss_ptr, grad_ptr))


def dp_student_use(ctx, on: bool):
    return check(ctx, lib().dp_student_use(ctx, int(bool(on))))


def dp_student_judge(ctx, every: int, max_force_rmse: float):
    return check(ctx, lib().dp_student_judge(ctx, int(every), float(max_force_rmse)))


def dp_student_judge_sample(ctx, side: float):
    return check(ctx, lib().dp_student_judge_sample(ctx, float(side)))


def dp_student_get_model(ctx) -> bytes:
    n = C.c_size_t()
    check(ctx, lib().dp_student_get_model(ctx, None, 0, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    check(ctx, lib().dp_student_get_model(ctx, buf, n.value, C.byref(n)))
    return buf.raw[:n.value]


def dp_student_set_model(ctx, blob: bytes):
    return check(ctx, lib().dp_student_set_model(ctx, blob, len(blob)))


def dp_destroy(ctx):
    lib().dp_destroy(ctx)
