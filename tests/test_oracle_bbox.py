"""Pins for the oracle's bounding box (Sec. 2.3): hand fixtures and brute force."""

import numpy as np
import pytest

from conftest import parse_cases
from oracle.bbox import bbox_from_cells


@pytest.mark.parametrize("case", parse_cases("bbox_cases.txt"), ids=lambda c: c["name"])
def test_hand_derived(case):
    nx, ny, nz = (int(v) for v in case["dims"])
    cell = np.zeros((nz, ny, nx), np.int32)
    for i, t in enumerate(case.get("cells", [])):
        x, y, z = (int(v) for v in t.split(","))
        cell[z, y, x] = i + 1
    got = bbox_from_cells(cell, int(case["margin"][0]))
    if "none" in case:
        assert got is None
    else:
        assert got == (tuple(int(v) for v in case["lo"]), tuple(int(v) for v in case["hi"]))


@pytest.mark.parametrize("seed", range(6))
def test_brute_force(seed):
    """Compare with a per-voxel Python loop that tracks the extremes directly."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = rng.integers(3, 12, size=3)
    cell = np.where(rng.random((nz, ny, nx)) < rng.uniform(0.002, 0.05),
                    rng.integers(1, 50, (nz, ny, nx)), 0).astype(np.int32)
    if seed == 0:
        cell[:] = 0
        cell[nz - 1, 0, nx // 2] = 3
    margin = int(rng.integers(0, 5))
    lo = [10 ** 9] * 3
    hi = [-1] * 3
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if cell[z, y, x] > 0:
                    for d, v in enumerate((x, y, z)):
                        lo[d] = min(lo[d], v)
                        hi[d] = max(hi[d], v)
    got = bbox_from_cells(cell, margin)
    if hi[0] < 0:
        assert got is None
        return
    n = (nx, ny, nz)
    want = (tuple(max(lo[d] - margin, 0) for d in range(3)),
            tuple(min(hi[d] + margin + 1, n[d]) for d in range(3)))
    assert got == want


def test_negative_cell_ids_are_not_cells():
    cell = np.zeros((4, 4, 4), np.int32)
    cell[1, 1, 1] = -5
    assert bbox_from_cells(cell, 1) is None
