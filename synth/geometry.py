"""Synthetic geometries and coefficient fields (data only, no solver arithmetic).

The paper's domain comes from segmented CT scans and a cellular Potts model
(Sec. 2.1, Fig. 2).  Neither is available, so each workload is replaced by a
seeded stand-in with the same structure:

* the pleural space is the shell between two nested ellipsoids per lung;
* tumour cells are Voronoi regions of seeds drawn inside that shell;
* per-species coefficients follow the generic linear reaction-diffusion form
  (diffusivity D, first-order uptake/decay k, production s).

All arrays are C-ordered ``[z][y][x]``; sizes and coordinates are ``(x, y, z)``.
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np
from scipy.spatial import cKDTree

Vec3 = Tuple[int, int, int]


@dataclasses.dataclass
class Problem:
    """One lattice with its domain mask, tumour cells and species coefficients."""

    name: str
    dims: Vec3                      # lattice size (nx, ny, nz)
    mask: np.ndarray                # uint8 [nz][ny][nx]; 1 = inside the simulated domain
    cell_id: np.ndarray             # int32 [nz][ny][nx]; 0 = no tumour cell, else cell index + 1
    D: np.ndarray                   # float64 [S][nz][ny][nx] diffusivity
    k: np.ndarray                   # float64 [S][nz][ny][nx] first-order uptake / decay rate
    src: np.ndarray                 # float64 [S][nz][ny][nx] production rate
    c0: np.ndarray                  # float64 [S][nz][ny][nx] initial concentrations
    c_b: np.ndarray                 # float64 [S] Dirichlet value on box faces
    dt: float = 1.0
    h: float = 1.0
    margin: int = 4
    box: Optional[Tuple[Vec3, Vec3]] = None   # fixed half-open box (lo, hi); None = from cells
    steps: int = 1
    tol: float = 1e-8

    @property
    def nspecies(self) -> int:
        return int(self.D.shape[0])

    def copy(self) -> "Problem":
        return dataclasses.replace(
            self,
            mask=self.mask.copy(), cell_id=self.cell_id.copy(), D=self.D.copy(),
            k=self.k.copy(), src=self.src.copy(), c0=self.c0.copy(), c_b=self.c_b.copy())


def _centres(dims: Vec3):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij", sparse=True)
    return x, y, z


def _inside_ellipsoid(dims: Vec3, centre, semi) -> np.ndarray:
    x, y, z = _centres(dims)
    cx, cy, cz = centre
    ax, ay, az = semi
    return ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((z - cz) / az) ** 2 <= 1.0


def dilate6(region: np.ndarray, allowed: Optional[np.ndarray] = None) -> np.ndarray:
    """One step of 6-neighbour binary dilation, optionally restricted to ``allowed``."""
    out = region.copy()
    out[1:, :, :] |= region[:-1, :, :]
    out[:-1, :, :] |= region[1:, :, :]
    out[:, 1:, :] |= region[:, :-1, :]
    out[:, :-1, :] |= region[:, 1:, :]
    out[:, :, 1:] |= region[:, :, :-1]
    out[:, :, :-1] |= region[:, :, 1:]
    if allowed is not None:
        out &= allowed
    return out


def voronoi_labels(points: np.ndarray, seeds: np.ndarray) -> np.ndarray:
    """Label each integer point with its nearest seed (squared integer distance).

    Ties go to the lowest seed index.  Returns int32 labels in ``[0, len(seeds))``.
    """
    kq = min(8, len(seeds))
    tree = cKDTree(seeds.astype(np.float64))
    _, cand = tree.query(points.astype(np.float64), k=kq)
    cand = cand.reshape(len(points), kq)
    diff = points[:, None, :].astype(np.int64) - seeds[cand].astype(np.int64)
    d2 = (diff * diff).sum(axis=2)
    # lexicographic (distance, seed index) minimum among the candidates
    key = d2 * np.int64(len(seeds) + 1) + cand
    best = np.argmin(key, axis=1)
    return cand[np.arange(len(points)), best].astype(np.int32)


def _species_fields(dims: Vec3, mask, tumour, rng, *, D, k_cell, k_all, s_cell,
                    D_tumour_factor=1.0, jitter=0.2, coef_scale=None):
    """Per-species D, k, s following the generic form dc/dt = div(D grad c) - k c + s.

    ``k_cell`` applies on tumour voxels, ``k_all`` on every voxel (decay), ``s_cell``
    is produced on tumour voxels.  k on tumour voxels is multiplied by an independent
    U(1-jitter, 1+jitter) factor per (species, voxel).
    """
    nx, ny, nz = dims
    S = len(D)
    shape = (S, nz, ny, nx)
    Df = np.empty(shape)
    kf = np.zeros(shape)
    sf = np.zeros(shape)
    ncell = int(tumour.sum())
    scale = np.ones((3, S)) if coef_scale is None else coef_scale
    for s in range(S):
        Df[s] = D[s] * scale[0, s]
        if D_tumour_factor != 1.0:
            Df[s][tumour] *= D_tumour_factor
        kf[s] = k_all[s] * scale[1, s]
        kt = (k_cell[s] + k_all[s]) * scale[1, s]
        if jitter > 0.0:
            kt = kt * rng.uniform(1.0 - jitter, 1.0 + jitter, size=ncell)
        kf[s][tumour] = kt
        sf[s][tumour] = s_cell[s] * scale[2, s]
    del mask
    return Df, kf, sf


# Species constants shared by the lung workloads: (oxygen, nutrient, cytokine).
LUNG_D = (1.0, 0.6, 0.3)
LUNG_K_CELL = (0.05, 0.02, 0.0)
LUNG_K_ALL = (0.0, 0.0, 0.005)
LUNG_S_CELL = (0.0, 0.0, 0.01)
LUNG_CB = (1.0, 1.0, 0.0)

# Four-species variant: the paper's two interleukins as separate fields instead of one
# cytokine field (oxygen, nutrient, IL-6, IL-8), each decaying everywhere and produced
# on tumour voxels.  The values are synthetic: the paper gives none.
LUNG4_D = (1.0, 0.6, 0.3, 0.25)
LUNG4_K_CELL = (0.05, 0.02, 0.0, 0.0)
LUNG4_K_ALL = (0.0, 0.0, 0.005, 0.004)
LUNG4_S_CELL = (0.0, 0.0, 0.01, 0.008)
LUNG4_CB = (1.0, 1.0, 0.0, 0.0)


def species_constants(nspecies: int = 3):
    """(D, k_cell, k_all, s_cell, c_b) of the 3-species or 4-species set."""
    if nspecies == 3:
        return LUNG_D, LUNG_K_CELL, LUNG_K_ALL, LUNG_S_CELL, LUNG_CB
    if nspecies == 4:
        return LUNG4_D, LUNG4_K_CELL, LUNG4_K_ALL, LUNG4_S_CELL, LUNG4_CB
    raise ValueError("species sets exist for 3 and 4 species")


def config1() -> Problem:
    """32^3 box, all voxels in the domain, one species (oxygen).

    Sphere of radius 8 voxels centred in the box, tested in integer arithmetic on
    doubled voxel-centre coordinates: (2i-31)^2 + (2j-31)^2 + (2k-31)^2 <= 256.
    D = 0.5 inside / 1.0 outside, uptake k = 0.1 inside / 0 outside, no source,
    Dirichlet c = 1 on the box faces, initial c = 1, dt = 1, 10 steps, tol 1e-10.
    """
    n = 32
    i = np.arange(n)
    zz, yy, xx = np.meshgrid(i, i, i, indexing="ij")
    sphere = (2 * xx - 31) ** 2 + (2 * yy - 31) ** 2 + (2 * zz - 31) ** 2 <= 256
    D = np.where(sphere, 0.5, 1.0)[None].astype(np.float64)
    k = np.where(sphere, 0.1, 0.0)[None].astype(np.float64)
    src = np.zeros_like(D)
    c0 = np.ones_like(D)
    mask = np.ones((n, n, n), np.uint8)
    cell = sphere.astype(np.int32)
    return Problem("config1", (n, n, n), mask, cell, D, k, src, c0, np.array([1.0]),
                   box=((0, 0, 0), (n, n, n)), steps=10, tol=1e-10)


def _lung_lattice(dims: Vec3, centres, outer, thickness):
    shell = np.zeros(dims[::-1], bool)
    for c in centres:
        inner = tuple(a - thickness for a in outer)
        shell |= _inside_ellipsoid(dims, c, outer) & ~_inside_ellipsoid(dims, c, inner)
    return shell


def _lung_problem(name, dims, centres, outer, window_lo, window_hi, ncells, seed,
                  steps, tol, thickness=6, dense=False, species=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    shell = _lung_lattice(dims, centres, outer, thickness)
    nx, ny, nz = dims
    win = np.zeros_like(shell)
    (x0, y0, z0), (x1, y1, z1) = window_lo, window_hi
    win[z0:z1, y0:y1, x0:x1] = True
    cand = np.argwhere(shell & win)               # (z, y, x) in C order
    pick = np.sort(rng.choice(len(cand), size=ncells, replace=False))
    seeds = cand[pick]
    labels = voronoi_labels(cand, seeds)
    cell = np.zeros(shell.shape, np.int32)
    cell[cand[:, 0], cand[:, 1], cand[:, 2]] = labels + 1
    tumour = cell > 0
    Dc, kc, ka, sc, cb = species_constants(species)
    D, k, s = _species_fields(dims, shell, tumour, rng, D=Dc, k_cell=kc, k_all=ka, s_cell=sc)
    c0 = np.broadcast_to(np.array(cb)[:, None, None, None], D.shape).copy()
    mask = np.ones_like(shell, dtype=np.uint8) if dense else shell.astype(np.uint8)
    return Problem(name, dims, mask, cell, D, k, s, c0, np.array(cb),
                   steps=steps, tol=tol)


def config2(seed: int = 20250503, dense: bool = False, species: int = 3) -> Problem:
    """256x256x160 lattice, pleural shell (6 voxels) of two ellipsoidal lungs.

    4000 tumour cells: Voronoi regions of seeds drawn without replacement from the
    shell voxels of the window x in [6,126), y in [64,184), z in [8,128).  The
    cell extent is the window, so with margin 4 the box is 128^3.  Three species,
    k on tumour voxels jittered by U(0.8, 1.2), 50 steps at dt = 1, tol 1e-8.
    ``species=4`` splits the cytokine into IL-6 and IL-8.
    """
    name = ("config2-dense" if dense else "config2") + ("-s4" if species == 4 else "")
    return _lung_problem(name, (256, 256, 160),
                         [(66, 128, 80), (190, 128, 80)], (60, 120, 76),
                         (6, 64, 8), (126, 184, 128), 4000, seed, 50, 1e-8, dense=dense,
                         species=species)


def config2_dense(seed: int = 20250503, species: int = 3) -> Problem:
    """config2 with every lattice voxel in the domain (same cells and coefficients)."""
    return config2(seed, dense=True, species=species)


def config5(seed: int = 20250503, species: int = 3) -> Problem:
    """512x512x320 lattice, two lungs, 60000 cells; box 384x384x256 (margin 4)."""
    return _lung_problem("config5" + ("-s4" if species == 4 else ""), (512, 512, 320),
                         [(132, 256, 160), (380, 256, 160)],
                         (120, 240, 152), (12, 68, 8), (388, 444, 256), 60000, seed,
                         100, 1e-8, species=species)


def cube(n: int, species: int = 3, seed: int = 2505) -> Problem:
    """Dense n^3 box, every voxel in the domain: the mesh-size sweep (n = 100, 150, 200).

    The box is the whole lattice.  The tumour is the ellipsoid with semi-axes
    (0.30 n, 0.25 n, 0.20 n) centred in the box, split into Voronoi cells of about 50
    voxels; D is halved and k applies (jittered) on tumour voxels, as in the growing
    tumour workload.  50 steps at dt = 1, tol 1e-8.
    """
    dims = (n, n, n)
    rng = np.random.Generator(np.random.PCG64(seed + n))
    tumour = _inside_ellipsoid(dims, (n / 2, n / 2, n / 2), (0.30 * n, 0.25 * n, 0.20 * n))
    pts = np.argwhere(tumour)
    nseed = max(1, len(pts) // 50)
    seeds = pts[np.sort(rng.choice(len(pts), size=nseed, replace=False))]
    labels = voronoi_labels(pts, seeds)
    mask = np.ones((n, n, n), np.uint8)
    prob = _tumour_problem(f"cube{n}" + ("-s4" if species == 4 else ""), dims, mask, tumour, rng,
                           species=species)
    prob.cell_id[pts[:, 0], pts[:, 1], pts[:, 2]] = labels + 1
    prob.box = ((0, 0, 0), dims)
    prob.steps = 50
    return prob


def config3_tumour(t: int) -> Tuple[Problem, np.ndarray]:
    """Tumour t of the 8-tumour growing-box workload (all voxels in the domain).

    Ellipsoid semi-axes (a, a, c), a = 28 + round(44 t / 7), c = 28 + round(12 t / 7),
    centred on the lattice midpoint (a voxel corner).  The lattice is the final box
    (after 20 one-voxel dilations, margin 4) plus 16 voxels per axis.  Returns the
    problem at step 0 and the boolean tumour region; the driver dilates it.
    """
    a = 28 + int(round(44 * t / 7))
    c = 28 + int(round(12 * t / 7))
    final = (2 * a + 40 + 8, 2 * a + 40 + 8, 2 * c + 40 + 8)
    dims = tuple(f + 16 for f in final)
    mid = tuple(d / 2 for d in dims)
    tumour = _inside_ellipsoid(dims, mid, (a, a, c))
    rng = np.random.Generator(np.random.PCG64(t + 1))
    mask = np.ones(dims[::-1], np.uint8)
    prob = _tumour_problem(f"config3-t{t}", dims, mask, tumour, rng)
    prob.steps = 200
    return prob, tumour


def _tumour_problem(name, dims, mask, tumour, rng, coef_scale=None, jitter=0.2, species=3):
    Dc, kc, ka, sc, cb = species_constants(species)
    D, k, s = _species_fields(dims, mask, tumour, rng, D=Dc, k_cell=kc, k_all=ka, s_cell=sc,
                              D_tumour_factor=0.5, jitter=jitter, coef_scale=coef_scale)
    c0 = np.broadcast_to(np.array(cb)[:, None, None, None], D.shape).copy()
    return Problem(name, dims, mask, tumour.astype(np.int32), D, k, s, c0,
                   np.array(cb), steps=1, tol=1e-8)


def config4_patch(seed: int, n: int = 64) -> Problem:
    """One training/evaluation geometry for the learned warm start.

    n^3 box, all voxels active.  The tumour is a random ellipsoid (semi-axes
    U(6, 20) * n / 64, centre uniform with the ellipsoid inside the box) split into
    Voronoi cells of U{20..200} seeds.  Coefficients are the tumour-workload ones,
    each per-species coefficient scaled by U(0.5, 1.5) per patch.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    semi = rng.uniform(6.0, 20.0, size=3) * (n / 64.0)
    lo = semi + 1.0
    hi = n - semi - 1.0
    centre = rng.uniform(lo, hi)
    dims = (n, n, n)
    tumour = _inside_ellipsoid(dims, tuple(centre), tuple(semi))
    pts = np.argwhere(tumour)
    nseed = int(rng.integers(20, 201))
    nseed = min(nseed, len(pts))
    seeds = pts[np.sort(rng.choice(len(pts), size=nseed, replace=False))]
    labels = voronoi_labels(pts, seeds)
    scale = rng.uniform(0.5, 1.5, size=(3, 3))
    mask = np.ones((n, n, n), np.uint8)
    prob = _tumour_problem(f"config4-{seed}", dims, mask, tumour, rng, coef_scale=scale)
    prob.cell_id[pts[:, 0], pts[:, 1], pts[:, 2]] = labels + 1
    prob.box = ((0, 0, 0), dims)
    prob.steps = 50
    return prob


def fourier_box(dims: Vec3, S: int = 1, D=1.0, k=0.0, s=0.0, c_b=0.0, interior_only=False):
    """Uniform-coefficient box used by the closed-form tests.

    ``interior_only`` shrinks the domain mask by one voxel on every side so that
    no domain voxel touches a box face (zero-flux problem).
    """
    nx, ny, nz = dims
    shape = (S, nz, ny, nx)
    mask = np.ones((nz, ny, nx), np.uint8)
    if interior_only:
        mask[:] = 0
        mask[1:-1, 1:-1, 1:-1] = 1
    ones = np.ones(shape)
    cb = np.broadcast_to(np.asarray(c_b, float), (S,)).copy()
    return Problem("fourier", dims, mask, np.zeros((nz, ny, nx), np.int32),
                   ones * np.asarray(D, float).reshape(-1, 1, 1, 1) if np.ndim(D) else ones * D,
                   ones * np.asarray(k, float).reshape(-1, 1, 1, 1) if np.ndim(k) else ones * k,
                   ones * np.asarray(s, float).reshape(-1, 1, 1, 1) if np.ndim(s) else ones * s,
                   np.broadcast_to(cb[:, None, None, None], shape).copy(), cb,
                   box=((0, 0, 0), dims))


def random_problem(seed: int, dims: Vec3, S: int = 3, fill: float = 0.6,
                   box: Optional[Tuple[Vec3, Vec3]] = None, dt: float = 1.0,
                   h: float = 1.0, smooth: int = 2) -> Problem:
    """Random masked lattice with random positive coefficients (parity-test input).

    The mask is a thresholded, box-filtered random field so that it has holes,
    ragged rows and isolated voxels.  D in [0.2, 2], k in [0, 0.2] (zero on a random
    third of voxels), s in [0, 0.05], c0 in [0, 1].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    f = rng.random((nz, ny, nx))
    for _ in range(smooth):
        f = (f + np.roll(f, 1, 0) + np.roll(f, 1, 1) + np.roll(f, 1, 2)) / 4.0
    thr = np.quantile(f, 1.0 - fill)
    mask = (f >= thr).astype(np.uint8)
    shape = (S, nz, ny, nx)
    D = rng.uniform(0.2, 2.0, shape)
    k = rng.uniform(0.0, 0.2, shape) * (rng.random(shape) > 0.33)
    src = rng.uniform(0.0, 0.05, shape)
    c0 = rng.uniform(0.0, 1.0, shape)
    cb = rng.uniform(0.0, 1.0, S)
    cell = (rng.random((nz, ny, nx)) < 0.05).astype(np.int32)
    if box is None:
        box = ((0, 0, 0), dims)
    return Problem(f"random-{seed}", dims, mask, cell, D, k, src, c0, cb, dt=dt, h=h,
                   box=box)


def tumour_coefficients(tumour: np.ndarray, jitter: np.ndarray):
    """D, k, s of the three lung species for a given tumour region (tumour workloads).

    D halves inside the tumour; k (uptake on tumour voxels, decay everywhere) is
    multiplied on tumour voxels by ``jitter[s]`` (an array drawn once per lattice, so
    that a growing tumour keeps the same factors where it already was).
    """
    S = 3
    shape = (S,) + tumour.shape
    D = np.empty(shape)
    k = np.empty(shape)
    s = np.zeros(shape)
    for sp in range(S):
        D[sp] = np.where(tumour, 0.5 * LUNG_D[sp], LUNG_D[sp])
        k[sp] = np.where(tumour, (LUNG_K_CELL[sp] + LUNG_K_ALL[sp]) * jitter[sp], LUNG_K_ALL[sp])
        s[sp] = np.where(tumour, LUNG_S_CELL[sp], 0.0)
    return D, k, s


@dataclasses.dataclass
class Growth:
    """Changes of one growth step: voxels taken by tumour cells and their new values."""

    index: np.ndarray     # int64 [n] flat lattice indices (C order)
    cell: np.ndarray      # int32 [n] new cell_id
    k: np.ndarray         # float64 [S][n] new k
    src: np.ndarray       # float64 [S][n] new production rate


def grow_cells(prob: Problem, steps: int, frac: float = 0.01, seed: int = 7) -> list:
    """Cell growth of the lung workloads, one list entry per step.

    Each step a seeded ``frac`` of the cells (drawn without replacement) each take one
    domain voxel that is 6-adjacent to the cell and not yet tumour, chosen uniformly
    among the candidates of that cell (a cell without candidates does not grow; two
    cells that pick the same voxel: the lower index wins).  The taken voxel gets the
    cell's species coefficients: k_cell + k_all jittered by U(0.8, 1.2) per species,
    and the production s_cell.  ``prob`` is not modified.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    _, kc, ka, sc, _ = species_constants(prob.nspecies)
    nz, ny, nx = prob.cell_id.shape
    cell = prob.cell_id.reshape(-1).copy()
    dom = prob.mask.reshape(-1) != 0
    ncell = int(cell.max())
    # voxels of each cell, kept as growing lists
    order = np.argsort(cell, kind="stable")
    first = np.searchsorted(cell[order], np.arange(1, ncell + 2))
    members = [list(order[first[i]:first[i + 1]]) for i in range(ncell)]
    out = []
    for _ in range(steps):
        pick = np.sort(rng.choice(ncell, size=max(1, int(round(frac * ncell))), replace=False))
        taken = {}
        for c in pick:
            v = np.asarray(members[c], np.int64)
            x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
            cand = []
            for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                xx, yy, zz = x + dx, y + dy, z + dz
                ok = (xx >= 0) & (xx < nx) & (yy >= 0) & (yy < ny) & (zz >= 0) & (zz < nz)
                cand.append(((zz * ny + yy) * nx + xx)[ok])
            cand = np.unique(np.concatenate(cand))
            cand = cand[dom[cand] & (cell[cand] == 0)]
            cand = [u for u in cand.tolist() if u not in taken]
            if not cand:
                continue
            taken[cand[int(rng.integers(len(cand)))]] = int(c) + 1
        idx = np.fromiter(taken.keys(), np.int64, len(taken))
        ids = np.fromiter(taken.values(), np.int32, len(taken))
        for u, c in zip(idx.tolist(), ids.tolist()):
            cell[u] = c
            members[c - 1].append(u)
        S = prob.nspecies
        k = np.empty((S, len(idx)))
        s = np.empty((S, len(idx)))
        for sp in range(S):
            k[sp] = (kc[sp] + ka[sp]) * rng.uniform(0.8, 1.2, size=len(idx))
            s[sp] = sc[sp]
        out.append(Growth(idx, ids, k, s))
    return out
