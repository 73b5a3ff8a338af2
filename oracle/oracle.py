"""ctypes wrapper of the FP64 CPU oracle (dp_oracle.c) -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It imports nothing from the HIP package; it takes plain numpy arrays
and a model blob (bytes) and returns numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "dp_oracle.c")


def build(force: bool = False) -> str:
    """Compile dp_oracle.c with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        i64 = C.c_int64
        L.or_model_new.restype = P
        L.or_model_new.argtypes = [C.c_char_p, i64]
        L.or_model_free.argtypes = [P]
        L.or_model_dims.argtypes = [P, P]
        L.or_last_error.restype = C.c_char_p
        L.or_wrap.argtypes = [i64, P, P, P]
        L.or_nlist.argtypes = [P, i64, P, P, P, P, i64, C.c_int, P, P, P]
        L.or_env_single.argtypes = [P, P, P, P]
        L.or_embed_single.argtypes = [P, C.c_int, C.c_int, C.c_double, P]
        L.or_eval.argtypes = [P, i64, P, P, P, P, i64, C.c_int, P, P, P, P, P, P, P, P, P, P, P, P]
        L.or_verlet.argtypes = [P, i64, P, P, P, P, P, C.c_double, i64, i64, C.c_int, P]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """FP64 reference evaluator for one model blob."""

    def __init__(self, blob: bytes):
        L = lib()
        self._blob = bytes(blob)
        self.h = L.or_model_new(self._blob, len(self._blob))
        if not self.h:
            raise ValueError("oracle: " + L.or_last_error().decode())
        d = np.zeros(6, dtype=np.int64)
        L.or_model_dims(self.h, _p(d))
        self.ntypes, self.n_emb, self.n_fit, self.M1, self.M2, self.nnei = (int(v) for v in d)

    def __del__(self):
        try:
            if self.h:
                lib().or_model_free(self.h)
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise ValueError(f"oracle error {rc}: " + lib().or_last_error().decode())

    def nlist(self, coords, types, box, centres=None, use_cells=True):
        x, b = _f64(coords), _f64(box)
        t = np.ascontiguousarray(types, dtype=np.int32)
        n = x.shape[0]
        c = None if centres is None else np.ascontiguousarray(centres, dtype=np.int64)
        nc = n if c is None else c.size
        nl = np.empty((nc, self.nnei), dtype=np.int32)
        nr = np.empty((nc, self.ntypes), dtype=np.int32)
        ovf = np.zeros(1, dtype=np.int64)
        self._check(lib().or_nlist(self.h, n, _p(x), _p(t), _p(b), _p(c), nc, int(use_cells), _p(nl),
                                   _p(nr), _p(ovf)))
        return nl, nr, int(ovf[0])

    def env_single(self, d):
        d = _f64(d)
        R = np.empty(4)
        J = np.empty((4, 3))
        lib().or_env_single(self.h, _p(d), _p(R), _p(J))
        return R, J

    def embed(self, t, u, s):
        G = np.empty(self.M1)
        lib().or_embed_single(self.h, int(t), int(u), float(s), _p(G))
        return G

    def eval(self, coords, types, box, centres=None, nthreads=0, intermediates=False):
        """Returns dict(energy, force[N,3], virial[3,3], atom_e, overflow, ...)."""
        x, b = _f64(coords), _f64(box)
        t = np.ascontiguousarray(types, dtype=np.int32)
        n = x.shape[0]
        c = None if centres is None else np.ascontiguousarray(centres, dtype=np.int64)
        nc = n if c is None else c.size
        e = np.zeros(1)
        f = np.zeros((n, 3))
        v = np.zeros(9)
        ae = np.zeros(nc)
        ovf = np.zeros(1, dtype=np.int64)
        out = dict()
        if intermediates:
            out["nlist"] = np.empty((nc, self.nnei), dtype=np.int32)
            out["nreal"] = np.empty((nc, self.ntypes), dtype=np.int32)
            out["rt"] = np.zeros((nc, self.nnei, 4))
            out["T"] = np.zeros((nc, self.M1, 4))
            out["D"] = np.zeros((nc, self.M1 * self.M2))
            out["dD"] = np.zeros((nc, self.M1 * self.M2))
            out["net_deriv"] = np.zeros((nc, self.nnei, 4))
        g = out.get
        self._check(lib().or_eval(self.h, n, _p(x), _p(t), _p(b), _p(c), nc, int(nthreads), _p(e), _p(f),
                                  _p(v), _p(ae), _p(g("nlist")), _p(g("nreal")), _p(g("rt")), _p(g("T")),
                                  _p(g("D")), _p(g("dD")), _p(g("net_deriv")), _p(ovf)))
        out.update(energy=float(e[0]), force=f, virial=v.reshape(3, 3), atom_e=ae, overflow=int(ovf[0]))
        return out

    def verlet(self, coords, vel, types, box, masses, dt, nsteps, every=1, nthreads=0):
        x = _f64(coords).copy()
        v = _f64(vel).copy()
        t = np.ascontiguousarray(types, dtype=np.int32)
        th = np.zeros((nsteps // every + 1, 6)) if every > 0 else None
        self._check(lib().or_verlet(self.h, x.shape[0], _p(x), _p(v), _p(t), _p(_f64(box)), _p(_f64(masses)),
                                    float(dt), int(nsteps), int(every), int(nthreads), _p(th)))
        return x, v, th
