"""Finite-volume assembly of one implicit-Euler step (Sec. 2.2 eqs. 1-4, Sec. 2.4).

TEST INFRASTRUCTURE ONLY (see the package header).

Each species obeys the linear form dc/dt = div(D grad c) - k c + s, which covers
eqs. 1-2 (consumption S read as first-order uptake k c) and eqs. 3-4
(degradation mu c), plus an explicit production s.  The box is discretised by
cell-centred finite volumes on a uniform mesh of spacing h and advanced with
first-order implicit Euler (Sec. 2.4):

    (c^{n+1}_P - c^n_P) / dt = sum_f G_f (c^{n+1}_Q - c^{n+1}_P) - k_P c^{n+1}_P + s_P

with one flux term per face f of voxel P:

* neighbour Q in the box and in the domain: G_f = D_f / h^2, with the harmonic
  mean D_f = 2 D_P D_Q / (D_P + D_Q) (0 when D_P + D_Q = 0);
* neighbour Q in the box but outside the domain mask: no flux (G_f = 0);
* face on the box boundary: Dirichlet value c_b on the face, half a voxel from
  the centre, so G_f = 2 D_P / h^2 and c_Q is replaced by c_b.

Collecting terms gives the linear system A c^{n+1} = b with

    A_PP = 1 + dt k_P + dt sum_f G_f,     A_PQ = -dt G_f,
    b_P  = c^n_P + dt s_P + dt sum_{Dirichlet f} G_f c_b.

Pinned by (``tests/test_oracle_fv.py``): the hand-derived single-voxel and
two-voxel fixtures in ``tests/golden/fv_cases.txt``; exact per-step decay of
discrete sine (Dirichlet) and cosine (zero-flux) Fourier modes; mass
conservation; the discrete maximum principle; a constant state; the two-material
slab whose piecewise-linear steady profile only the harmonic mean preserves;
symmetry and M-matrix structure of A.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def harmonic_mean(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """2ab/(a+b), defined as 0 where a + b = 0."""
    s = a + b
    out = np.zeros(np.broadcast(a, b).shape)
    nz = s != 0
    out[nz] = (2.0 * a * b)[nz] / s[nz]
    return out


def box_slice(box):
    (x0, y0, z0), (x1, y1, z1) = box
    return (slice(z0, z1), slice(y0, y1), slice(x0, x1))


def active_index(mask_box: np.ndarray) -> np.ndarray:
    """Compact index of every in-domain voxel of the box, in C order; -1 elsewhere."""
    act = mask_box.astype(bool)
    idx = np.full(act.shape, -1, np.int64)
    idx[act] = np.arange(int(act.sum()))
    return idx


def assemble(mask_box, D_box, k_box, s_box, c_b: float, dt: float, h: float):
    """Assemble one species on the box: returns ``(A, q)``.

    ``A`` is the CSR matrix over the domain voxels of the box (C-order compact
    numbering, see ``active_index``) and ``q = dt s + dt sum_{Dirichlet} G c_b``,
    so that ``b = c^n + q``.
    """
    act = mask_box.astype(bool)
    idx = active_index(act)
    n = int(act.sum())
    P = np.argwhere(act)                                    # (z, y, x) rows
    D_P = D_box[act]
    diag = 1.0 + dt * k_box[act]
    q = dt * s_box[act]
    rows, cols, vals = [], [], []
    shape = np.array(act.shape)
    inv_h2 = 1.0 / (h * h)
    for axis in range(3):
        for step in (-1, 1):
            Q = P.copy()
            Q[:, axis] += step
            outside = (Q[:, axis] < 0) | (Q[:, axis] >= shape[axis])
            inside = ~outside
            Qi = Q[inside]
            q_active = np.zeros(n, bool)
            q_active[inside] = act[Qi[:, 0], Qi[:, 1], Qi[:, 2]]
            # Dirichlet box face: half-voxel distance to the face value
            G_dir = 2.0 * D_P[outside] * inv_h2
            diag[outside] += dt * G_dir
            q[outside] += dt * G_dir * c_b
            # interior face between two domain voxels: harmonic-mean diffusivity
            rP = np.nonzero(q_active)[0]
            Qa = Q[q_active]
            D_Q = D_box[Qa[:, 0], Qa[:, 1], Qa[:, 2]]
            G_int = harmonic_mean(D_P[rP], D_Q) * inv_h2
            diag[rP] += dt * G_int
            rows.append(rP)
            cols.append(idx[Qa[:, 0], Qa[:, 1], Qa[:, 2]])
            vals.append(-dt * G_int)
            # neighbour in the box but outside the mask: zero flux, nothing to add
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    A.sum_duplicates()
    return A, q


def gather(field, mask_box_bool, box):
    """Values of a lattice field ``[z][y][x]`` on the domain voxels of the box."""
    return field[box_slice(box)][mask_box_bool]
