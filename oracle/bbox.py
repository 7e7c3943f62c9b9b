"""Bounding box of all tumour cells plus a margin (Sec. 2.3).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper restricts the PDE domain to the bounding coordinates of all tumour
cells, widened by a margin to leave room for diffusion.  Reading used here:
the box is half-open ``[lo, hi)`` per axis, clamped to the lattice, and a lattice
without any tumour voxel has no box.

Pinned by: hand-derived fixtures in ``tests/golden/bbox_cases.txt`` and brute
force over every voxel on random lattices (``tests/test_oracle_bbox.py``).
"""

from __future__ import annotations

import numpy as np


def bbox_from_cells(cell_id: np.ndarray, margin: int):
    """Return ``(lo, hi)`` in (x, y, z) order, or ``None`` if no voxel has a cell.

    ``cell_id`` is ``[z][y][x]``; a voxel belongs to a tumour cell when its id is
    positive.  Per axis d: lo_d = max(min_d - margin, 0) and
    hi_d = min(max_d + margin + 1, n_d).
    """
    if margin < 0:
        raise ValueError("margin must be non-negative")
    zyx = np.nonzero(cell_id > 0)
    if len(zyx[0]) == 0:
        return None
    nz, ny, nx = cell_id.shape
    coords = (zyx[2], zyx[1], zyx[0])          # x, y, z
    sizes = (nx, ny, nz)
    lo = tuple(int(max(int(c.min()) - margin, 0)) for c in coords)
    hi = tuple(int(min(int(c.max()) + margin + 1, n)) for c, n in zip(coords, sizes))
    return lo, hi
