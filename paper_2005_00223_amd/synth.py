"""Seeded synthetic inputs: structures, velocities and random model weights.

This module is shared by the HIP path's tests and benchmark and by the oracle's
tests. It holds none of the Deep Potential arithmetic: it only places atoms,
draws random numbers and serialises weights into the model blob format that
both sides parse with their own code.

Workloads (stand-ins for the paper's liquid water and FCC copper systems,
Section VI "Physical systems"; the trained models and AIMD data are not
available, so weights are random and seeded):

* water: oxygen on a simple-cubic grid, two hydrogens per oxygen at the
  TIP3P-like geometry (0.9572 A, 104.52 deg) in a random orientation, then
  Gaussian jitter on every atom, then wrapping into the periodic box.
* copper: FCC lattice of conventional cells (4 atoms each), Gaussian jitter,
  wrapping.
"""
from __future__ import annotations

import itertools
import struct
from dataclasses import dataclass, field

import numpy as np

BLOB_MAGIC = b"DPMIBLOB"
BLOB_VERSION = 1
BLOB_VERSION_LINEAR_OUT = 2   # adds the emb_out_linear flag

# Units: A, fs, amu, eV.  1 amu*A^2/fs^2 = 103.6427 eV.
MVV2E = 103.642696562
KB_EV = 8.617333262e-5
MASS = {"O": 15.999, "H": 1.008, "Cu": 63.546}


# --------------------------------------------------------------------------
# structures
# --------------------------------------------------------------------------
def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation matrix from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _wrap(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    x = x - box * np.floor(x / box)
    x[x >= box] = 0.0
    return x


def water_system(n_side, box_len, jitter=0.1, seed=0, reps=(1, 1, 1)):
    """n_side^3 molecules on a simple-cubic grid in a cube of side box_len.

    ``reps`` tiles the cell (e.g. (2,1,1) doubles it along x) before jitter.
    Atom order is molecule by molecule (O, H, H); types O=0, H=1.
    Returns (coords [N,3] f64, types [N] i32, box [3] f64).
    """
    rng = np.random.default_rng(seed)
    a = box_len / n_side
    g = np.arange(n_side) * a + 0.5 * a
    ox = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    reps = tuple(int(r) for r in reps)
    shifts = np.stack(np.meshgrid(*[np.arange(r) for r in reps], indexing="ij"), -1).reshape(-1, 3)
    ox = (ox[None, :, :] + shifts[:, None, :] * box_len).reshape(-1, 3)
    box = np.array(reps, dtype=np.float64) * box_len
    roh, ang = 0.9572, np.deg2rad(104.52)
    h1 = roh * np.array([np.sin(ang / 2), np.cos(ang / 2), 0.0])
    h2 = roh * np.array([-np.sin(ang / 2), np.cos(ang / 2), 0.0])
    n_mol = ox.shape[0]
    coords = np.empty((3 * n_mol, 3))
    for m in range(n_mol):
        R = _random_rotation(rng)
        coords[3 * m] = ox[m]
        coords[3 * m + 1] = ox[m] + R @ h1
        coords[3 * m + 2] = ox[m] + R @ h2
    coords += rng.normal(scale=jitter, size=coords.shape)
    types = np.tile(np.array([0, 1, 1], dtype=np.int32), n_mol)
    return _wrap(coords, box), types, box


def fcc_copper(n_cells, a=3.634, jitter=0.05, seed=0):
    """n_cells^3 conventional FCC cells (4 atoms each), type 0 everywhere."""
    rng = np.random.default_rng(seed)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.arange(n_cells)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    coords = ((cells[:, None, :] + basis[None, :, :]) * a).reshape(-1, 3)
    if jitter > 0:
        coords = coords + rng.normal(scale=jitter, size=coords.shape)
    box = np.full(3, n_cells * a)
    return _wrap(coords, box), np.zeros(coords.shape[0], dtype=np.int32), box


def maxwell_boltzmann(masses, temp, seed):
    """Velocities (A/fs) at exactly ``temp`` K with 3N-3 degrees of freedom.

    Gaussian per component with variance kT/m, centre-of-mass momentum
    removed, then rescaled so that 2 KE / ((3N-3) k_B) == temp.
    """
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64)
    sig = np.sqrt(KB_EV * temp / (m * MVV2E))
    v = rng.normal(size=(m.size, 3)) * sig[:, None]
    p = (m[:, None] * v).sum(0) / m.sum()
    v -= p
    ke = 0.5 * MVV2E * (m[:, None] * v * v).sum()
    t_now = 2 * ke / ((3 * m.size - 3) * KB_EV)
    return v * np.sqrt(temp / t_now)


# --------------------------------------------------------------------------
# model
# --------------------------------------------------------------------------
@dataclass
class ModelSpec:
    ntypes: int
    rcut: float
    rcut_smth: float
    sel: tuple
    emb: tuple = (25, 50, 100)
    M2: int = 16
    fit: tuple = (240, 240, 240)
    desc_norm: float | None = None  # default: sum(sel)
    out_scale: float = 1.0
    seed: int = 0
    emb_W: list = field(default_factory=list)   # [t][u][l] -> (in,out)
    emb_b: list = field(default_factory=list)
    fit_W: list = field(default_factory=list)   # [t][l] -> (in,out); last is output
    fit_b: list = field(default_factory=list)
    emb_out_linear: bool = False   # last embedding layer without tanh

    @property
    def nnei(self):
        return int(sum(self.sel))

    @property
    def M1(self):
        return int(self.emb[-1])


def random_model(ntypes, rcut, rcut_smth, sel, emb=(25, 50, 100), M2=16,
                 fit=(240, 240, 240), seed=0, out_scale=1.0, desc_norm=None):
    """Xavier-normal weights (std sqrt(2/(fan_in+fan_out))), N(0,1) hidden
    biases, zero output bias, drawn with numpy default_rng(seed) in the order:
    embedding nets t-major, u, layer (W then b); then fitting nets t, layer.
    The output layer weight is multiplied by ``out_scale``."""
    rng = np.random.default_rng(seed)
    spec = ModelSpec(ntypes, float(rcut), float(rcut_smth), tuple(int(s) for s in sel),
                     tuple(int(e) for e in emb), int(M2), tuple(int(f) for f in fit),
                     float(desc_norm) if desc_norm else float(sum(sel)), float(out_scale), int(seed))
    widths = (1,) + spec.emb
    for t in range(ntypes):
        rowW, rowb = [], []
        for u in range(ntypes):
            Ws, bs = [], []
            for l in range(len(spec.emb)):
                fi, fo = widths[l], widths[l + 1]
                Ws.append(rng.normal(scale=np.sqrt(2.0 / (fi + fo)), size=(fi, fo)))
                bs.append(rng.normal(size=fo))
            rowW.append(Ws)
            rowb.append(bs)
        spec.emb_W.append(rowW)
        spec.emb_b.append(rowb)
    fw = (spec.M1 * spec.M2,) + spec.fit + (1,)
    for t in range(ntypes):
        Ws, bs = [], []
        for l in range(len(fw) - 1):
            fi, fo = fw[l], fw[l + 1]
            W = rng.normal(scale=np.sqrt(2.0 / (fi + fo)), size=(fi, fo))
            if l == len(fw) - 2:
                W = W * spec.out_scale
                b = np.zeros(fo)
            else:
                b = rng.normal(size=fo)
            Ws.append(W)
            bs.append(b)
        spec.fit_W.append(Ws)
        spec.fit_b.append(bs)
    return spec


def pack_blob(spec: ModelSpec) -> bytes:
    """Serialise to the DPMIBLOB layout (all little-endian):

    8 bytes magic "DPMIBLOB"; int64 version, ntypes, n_emb, n_fit, M2;
    version 2 only: int64 emb_out_linear (1 = the last embedding layer is
    affine, no tanh; version 1 means 0); float64 rcut, rcut_smth, desc_norm; int64 sel[ntypes];
    int64 emb_width[n_emb+1] (emb_width[0] == 1); int64 fit_width[n_fit];
    then float64 arrays: for t, for u, for embedding layer l: W[in][out]
    row-major, b[out]; then for t, for fitting layer l (n_fit hidden layers
    and the 1-wide output layer): W[in][out], b[out].
    """
    T = spec.ntypes
    head = BLOB_MAGIC
    ver = BLOB_VERSION_LINEAR_OUT if spec.emb_out_linear else BLOB_VERSION
    head += struct.pack("<5q", ver, T, len(spec.emb), len(spec.fit), spec.M2)
    if spec.emb_out_linear:
        head += struct.pack("<q", 1)
    head += struct.pack("<3d", spec.rcut, spec.rcut_smth, spec.desc_norm)
    head += struct.pack(f"<{T}q", *spec.sel)
    head += struct.pack(f"<{len(spec.emb) + 1}q", 1, *spec.emb)
    head += struct.pack(f"<{len(spec.fit)}q", *spec.fit)
    parts = [head]
    for t in range(T):
        for u in range(T):
            for W, b in zip(spec.emb_W[t][u], spec.emb_b[t][u]):
                parts.append(np.ascontiguousarray(W, dtype="<f8").tobytes())
                parts.append(np.ascontiguousarray(b, dtype="<f8").tobytes())
    for t in range(T):
        for W, b in zip(spec.fit_W[t], spec.fit_b[t]):
            parts.append(np.ascontiguousarray(W, dtype="<f8").tobytes())
            parts.append(np.ascontiguousarray(b, dtype="<f8").tobytes())
    return b"".join(parts)


STUDENT_H1, STUDENT_H2 = 16, 32


def student_np(M1: int) -> int:
    """Packed parameters per student net: W1[16] b1[16] W2[16][32] b2[32]
    W3[32][M1] b3[M1]."""
    return STUDENT_H1 * 2 + STUDENT_H1 * STUDENT_H2 + STUDENT_H2 + STUDENT_H2 * M1 + M1


def student_spec(teacher: ModelSpec, params) -> ModelSpec:
    """The teacher's geometry and fitting nets with student embedding nets
    1-16-32-M1 (affine last layer) taken from packed parameters
    params[t*ntypes+u] in the layout of student_np."""
    import copy
    T, M1 = teacher.ntypes, teacher.M1
    P = np.asarray(params, dtype=np.float64).reshape(T * T, student_np(M1))
    st = copy.deepcopy(teacher)
    st.emb = (STUDENT_H1, STUDENT_H2, M1)
    st.emb_out_linear = True
    h1, h2 = STUDENT_H1, STUDENT_H2
    cuts = np.cumsum([h1, h1, h1 * h2, h2, h2 * M1, M1])
    st.emb_W, st.emb_b = [], []
    for t in range(T):
        rw, rb = [], []
        for u in range(T):
            W1, b1, W2, b2, W3, b3 = np.split(P[t * T + u], cuts[:-1])
            rw.append([W1.reshape(1, h1), W2.reshape(h1, h2), W3.reshape(h2, M1)])
            rb.append([b1, b2, b3])
        st.emb_W.append(rw)
        st.emb_b.append(rb)
    return st


def random_student_params(teacher: ModelSpec, seed: int, w1_scale: float = 5.0):
    """Seeded random student parameters [ntypes^2][np] (float32 values):
    W1 ~ N(0, w1_scale^2), hidden biases N(0,1), W2 and W3 Xavier-normal,
    b3 N(0, 0.1^2)."""
    rng = np.random.default_rng(seed)
    T, M1 = teacher.ntypes, teacher.M1
    h1, h2 = STUDENT_H1, STUDENT_H2
    out = []
    for _ in range(T * T):
        out.append(np.concatenate([
            rng.normal(scale=w1_scale, size=h1), rng.normal(size=h1),
            rng.normal(scale=np.sqrt(2.0 / (h1 + h2)), size=h1 * h2), rng.normal(size=h2),
            rng.normal(scale=np.sqrt(2.0 / (h2 + M1)), size=h2 * M1), rng.normal(scale=0.1, size=M1)]))
    return np.array(out).astype(np.float32)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
# Descriptor constants Nc and output-layer scales, fixed once per system so
# that the random models have a descriptor of order one (the role DeePMD's
# environment statistics play for trained models) and an RMS force of about
# 1 eV/A on their own structures.  Random weights with Nc = sum(sel) and no
# output scale give RMS forces of 1e-5..1e-3 eV/A, which would make a 1e-3
# eV/A accuracy bar vacuous.  The sign is the one that gives the reference
# structure a positive virial trace (net repulsion): with the other sign both
# random models have no short-range repulsion at all and NVE trajectories
# collapse within 10-60 fs, while with this one 100-step NVE runs conserve
# the total energy (water 0.5 fs, copper 1 fs).
WATER_DESC_NORM, WATER_OUT_SCALE = 16.0, -8.0
CU_DESC_NORM, CU_OUT_SCALE = 8.0, -50.0


def water_model(seed=0, emb=(25, 50, 100)):
    return random_model(2, 6.0, 0.5, (46, 92), emb=emb, M2=16, fit=(240, 240, 240),
                        seed=seed, out_scale=WATER_OUT_SCALE, desc_norm=WATER_DESC_NORM)


def copper_model(seed=1, emb=(25, 50, 100)):
    return random_model(1, 8.0, 2.0, (512,), emb=emb, M2=16, fit=(240, 240, 240),
                        seed=seed, out_scale=CU_OUT_SCALE, desc_norm=CU_DESC_NORM)


def workload(name):
    """Return dict(coords, types, box, masses_per_type, spec, dt_fs, ...)."""
    if name == "water192":      # 64 molecules, 12.42 A
        x, t, box = water_system(4, 12.42, 0.1, seed=1)
        return dict(name=name, coords=x, types=t, box=box, masses=np.array([MASS["O"], MASS["H"]]),
                    spec=water_model(0), dt_fs=0.5, temp=300.0, vseed=101)
    if name == "water12288":    # 4,096 molecules, 49.7 A
        x, t, box = water_system(16, 49.7, 0.1, seed=2)
        return dict(name=name, coords=x, types=t, box=box, masses=np.array([MASS["O"], MASS["H"]]),
                    spec=water_model(0), dt_fs=0.5, temp=300.0, vseed=102)
    if name == "cu32000":       # 20^3 FCC cells
        x, t, box = fcc_copper(20, 3.634, 0.05, seed=3)
        return dict(name=name, coords=x, types=t, box=box, masses=np.array([MASS["Cu"]]),
                    spec=copper_model(1), dt_fs=1.0, temp=300.0, vseed=103)
    if name == "water24576":    # the 12,288-atom cell doubled along x
        x, t, box = water_system(16, 49.7, 0.1, seed=4, reps=(2, 1, 1))
        return dict(name=name, coords=x, types=t, box=box, masses=np.array([MASS["O"], MASS["H"]]),
                    spec=water_model(0), dt_fs=0.5, temp=300.0, vseed=104)
    if name == "cu13500":       # 15^3 FCC cells: the embedding-size sweep (Fig. 7) workload
        x, t, box = fcc_copper(15, 3.634, 0.05, seed=8)
        return dict(name=name, coords=x, types=t, box=box, masses=np.array([MASS["Cu"]]),
                    spec=copper_model(1), dt_fs=1.0, temp=300.0, vseed=108)
    if name == "cu500k":        # 50^3 FCC cells
        x, t, box = fcc_copper(50, 3.634, 0.05, seed=5)
        return dict(name=name, coords=x, types=t, box=box, masses=np.array([MASS["Cu"]]),
                    spec=copper_model(1), dt_fs=1.0, temp=300.0, vseed=105)
    if name.startswith("cu_cells"):  # cu_cellsN: N^3 FCC cells, jittered
        n = int(name[len("cu_cells"):])
        x, t, box = fcc_copper(n, 3.634, 0.05, seed=6)
        return dict(name=name, coords=x, types=t, box=box, masses=np.array([MASS["Cu"]]),
                    spec=copper_model(1), dt_fs=1.0, temp=300.0, vseed=106)
    raise KeyError(name)


def brick_share(coords, types, box, grid, brick, rc, pad=1.0):
    """One rank's share of a spatial decomposition of a periodic orthorhombic
    box into grid[0] x grid[1] x grid[2] bricks (Section V-D): the atoms whose
    wrapped position lies in brick `brick` (owned, first), then every atom or
    periodic image within rc of the brick (ghosts), translated into a box of
    the brick's size plus 2 rc + pad per axis, so that no periodic image of
    the local box comes within rc.  Pure geometry: no model arithmetic.

    Returns dict(coords [n,3], types [n], box [3], n_local, index [n] int32 =
    the atom each local atom is (ghosts: the atom they image))."""
    x = np.asarray(coords, dtype=np.float64)
    L = np.asarray(box, dtype=np.float64).reshape(-1)
    L = L if L.size == 3 else np.diag(L.reshape(3, 3))
    grid = np.asarray(grid, dtype=np.int64)
    b = np.asarray(brick, dtype=np.int64)
    side = L / grid
    if np.any(side <= 2.0 * rc):
        raise ValueError("bricks must be wider than 2 rc")
    xw = x - L * np.floor(x / L)
    lo, hi = b * side, (b + 1) * side
    cell = np.minimum(np.floor(xw / side).astype(np.int64), grid - 1)
    own = np.all(cell == b, axis=1)
    owned = np.nonzero(own)[0]
    gx, gi = [], []
    for s in itertools.product((-1, 0, 1), repeat=3):
        y = xw + np.asarray(s) * L
        inside = np.all((y >= lo - rc) & (y < hi + rc), axis=1)
        if s == (0, 0, 0):
            inside &= ~own
        sel = np.nonzero(inside)[0]
        gx.append(y[sel])
        gi.append(sel)
    gx = np.concatenate(gx)
    gi = np.concatenate(gi)
    shift = rc + 0.5 * pad - lo
    loc = np.concatenate([xw[owned], gx]) + shift
    return dict(coords=loc, types=np.concatenate([types[owned], types[gi]]).astype(np.int32),
                box=side + 2.0 * rc + pad, n_local=int(owned.size),
                index=np.concatenate([owned, gi]).astype(np.int32))
