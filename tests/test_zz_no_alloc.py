"""The entry point that allocates nothing (mpm_bbox_from_cells_noalloc) against the
allocating one (mpm_bbox_from_cells) and the oracle's brute-force box, called through
the C ABI: two calls in a row, the second on a smaller lattice, on the vector path
(nx a multiple of 4) and the scalar path, plus the empty lattice.  Boxes are integer
results, so the bar is bit-exact."""

import numpy as np
import pytest

from gpu_helpers import require_gpu
from oracle.bbox import bbox_from_cells

pytestmark = pytest.mark.gpu


def _lattice(dims, seed, npts):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    cell = np.zeros((nz, ny, nx), np.int32)
    pts = rng.integers(0, [nx, ny, nz], size=(npts, 3))
    cell[pts[:, 2], pts[:, 1], pts[:, 0]] = rng.integers(1, 1000, npts)
    return cell


@pytest.mark.parametrize("first,second", [((256, 256, 160), (64, 48, 40)),     # vector path
                                          ((255, 131, 97), (37, 29, 23))])      # scalar path
def test_noalloc_matches_allocating_entry_point(first, second):
    torch = require_gpu()
    from paper_2505_03067_amd import mpm_bbox_from_cells, mpm_bbox_from_cells_noalloc
    for i, dims in enumerate((first, second)):
        cell = _lattice(dims, seed=sum(dims) + i, npts=300)
        dev = torch.from_numpy(cell).cuda()
        for margin in (0, 4):
            got = mpm_bbox_from_cells_noalloc(dev, margin)
            ref = mpm_bbox_from_cells(dev, margin)
            want = bbox_from_cells(cell, margin)
            print(f"call {i} dims {dims} margin {margin}: noalloc {got} allocating {ref} oracle {want}",
                  flush=True)
            assert got == ref == want


def test_noalloc_empty_and_after_empty():
    """An empty lattice gives MPM_EEMPTY; the next call (smaller, one cell voxel) still
    finds its box, so nothing stale in the shared scratch leaks into a later result."""
    torch = require_gpu()
    from paper_2505_03067_amd import MPM_EEMPTY, MpmError, mpm_bbox_from_cells_noalloc
    big = np.zeros((40, 48, 64), np.int32)
    with pytest.raises(MpmError) as e:
        mpm_bbox_from_cells_noalloc(torch.from_numpy(big).cuda(), 2)
    assert e.value.code == MPM_EEMPTY
    small = np.zeros((5, 6, 7), np.int32)
    small[4, 0, 3] = 9
    got = mpm_bbox_from_cells_noalloc(torch.from_numpy(small).cuda(), 1)
    assert got == bbox_from_cells(small, 1) == ((2, 0, 3), (5, 2, 5))
