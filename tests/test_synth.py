"""The seeded input generators (CPU): determinism, the documented counts and the rules
of the cell-growth stand-in.  These hold no solver arithmetic; the tests check that the
inputs are what the workloads state."""

import numpy as np

from synth import config2, cube, species_constants
from synth.geometry import grow_cells


def test_config2_counts_and_determinism():
    a, b = config2(), config2()
    assert np.array_equal(a.cell_id, b.cell_id) and np.array_equal(a.k, b.k)
    assert a.dims == (256, 256, 160) and a.nspecies == 3
    # 4000 cells, box of the cells plus margin 4 is 128^3, 236,540 domain voxels in it
    assert a.cell_id.max() == 4000
    zyx = np.nonzero(a.cell_id > 0)
    lo = [max(int(v.min()) - 4, 0) for v in zyx[::-1]]
    hi = [min(int(v.max()) + 5, n) for v, n in zip(zyx[::-1], a.dims)]
    assert [h - l for l, h in zip(lo, hi)] == [128, 128, 128]
    box = tuple(slice(l, h) for l, h in zip(lo[::-1], hi[::-1]))
    assert int(a.mask[box].sum()) == 236540


def test_four_species_constants():
    D, kc, ka, sc, cb = species_constants(4)
    assert len(D) == len(kc) == len(ka) == len(sc) == len(cb) == 4
    # the two interleukins decay everywhere and are produced on tumour voxels only
    assert ka[2] > 0 and ka[3] > 0 and sc[2] > 0 and sc[3] > 0 and kc[2] == kc[3] == 0
    p = config2(species=4)
    assert p.nspecies == 4 and p.name == "config2-s4"
    tum = p.cell_id > 0
    assert np.all(p.src[3][~tum] == 0) and np.all(p.src[3][tum] == sc[3])


def test_cube_sweep_geometry():
    p = cube(40, species=3)
    assert p.dims == (40, 40, 40) and p.box == ((0, 0, 0), (40, 40, 40))
    assert p.mask.all()
    tum = p.cell_id > 0
    # D halved on the tumour, uptake jittered within +-20% there
    assert np.allclose(p.D[0][tum], 0.5) and np.allclose(p.D[0][~tum], 1.0)
    kt = p.k[0][tum] / 0.05
    assert kt.min() >= 0.8 - 1e-12 and kt.max() <= 1.2 + 1e-12
    # about 50 voxels per cell
    assert 30 <= tum.sum() / p.cell_id.max() <= 70


def test_grow_cells_rules():
    p = config2()
    steps = grow_cells(p, 6, seed=3)
    again = grow_cells(p, 6, seed=3)
    assert all(np.array_equal(a.index, b.index) and np.array_equal(a.k, b.k) for a, b in zip(steps, again))
    nz, ny, nx = p.cell_id.shape
    cell = p.cell_id.reshape(-1).copy()
    dom = p.mask.reshape(-1) != 0
    _, kc, ka, sc, _ = species_constants(3)
    grown = 0
    for st in steps:
        assert len(np.unique(st.index)) == len(st.index)            # one cell per voxel
        assert np.all(dom[st.index]) and np.all(cell[st.index] == 0)  # free domain voxels
        for u, c in zip(st.index.tolist(), st.cell.tolist()):
            x, y, z = u % nx, (u // nx) % ny, u // (nx * ny)
            nb = []
            for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                xx, yy, zz = x + dx, y + dy, z + dz
                if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                    nb.append(cell[(zz * ny + yy) * nx + xx])
            assert c in nb                                          # adjacent to its cell
        for s in range(3):
            lo, hi = (kc[s] + ka[s]) * 0.8, (kc[s] + ka[s]) * 1.2
            assert np.all(st.k[s] >= lo - 1e-15) and np.all(st.k[s] <= hi + 1e-15)
            assert np.all(st.src[s] == sc[s])
        cell[st.index] = st.cell
        grown += len(st.index)
    assert grown > 0
