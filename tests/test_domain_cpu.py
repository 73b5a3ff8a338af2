"""Host logic of the rank-share emulation (synth.brick_share), CPU only:
every atom is owned by exactly one brick, and every neighbour within rc of
an owned atom is present in its brick (as the owned atom or a ghost image)
at the right displacement, by brute force over periodic images."""
import itertools

import numpy as np

from paper_2005_00223_amd import synth


def _min_image_neighbours(x, L, i, rc):
    d = x - x[i]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(1))
    js = np.nonzero((r <= rc) & (np.arange(len(x)) != i))[0]
    return {(int(j), tuple(np.round(d[j], 9))) for j in js}


def test_bricks_partition_and_cover_neighbourhoods():
    x, t, box = synth.fcc_copper(6, 3.634, 0.05, seed=11)  # 864 atoms, 21.8 A
    L = np.asarray(box, dtype=np.float64)
    rc = 5.0
    owners = np.zeros(len(t), dtype=np.int64)
    rng = np.random.default_rng(0)
    for b in itertools.product(range(2), repeat=3):
        sh = synth.brick_share(x, t, L, (2, 2, 2), b, rc)
        nl = sh["n_local"]
        owners[sh["index"][:nl]] += 1
        assert np.array_equal(sh["types"], t[sh["index"]])
        y = sh["coords"]
        Lb = np.asarray(sh["box"])
        assert np.all(y >= 0) and np.all(y < Lb)
        for k in rng.choice(nl, size=min(nl, 12), replace=False):
            i = sh["index"][k]
            want = _min_image_neighbours(x, L, i, rc)
            d = y - y[k]
            r = np.sqrt((d ** 2).sum(1))
            got = {(int(sh["index"][m]), tuple(np.round(d[m], 9))) for m in np.nonzero((r <= rc) & (np.arange(len(y)) != k))[0]}
            assert got == want
            # no periodic image of the local box within rc of an owned atom
            dd = d - Lb * np.round(d / Lb)
            assert np.allclose(dd[r <= rc], d[r <= rc])
            far = np.sqrt((dd ** 2).sum(1))
            assert not np.any((far <= rc) & (r > rc))
    assert np.all(owners == 1)
