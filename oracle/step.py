"""One implicit-Euler step on the tumour bounding box (Sec. 2.3-2.4).

TEST INFRASTRUCTURE ONLY (see the package header).

The step as the paper describes it: take the box around the tumour cells plus a
margin (Sec. 2.3), discretise the domain inside the box by finite volumes and
advance one first-order implicit Euler step with an iterative solve (Sec. 2.4),
then write the result back onto the pleural mask (Sec. 2.4).  Voxels outside
the box or outside the mask keep their values.  Species are uncoupled within a
step (eqs. 1-4 have no cross terms), so each species is solved on its own.

Pinned through ``fv`` and ``krylov``; the whole step is additionally checked
by ``tests/test_oracle_step.py`` (Fourier decay after several steps, config-1
mirror symmetry, LU/PCG/GMRES agreement).
"""

from __future__ import annotations

import numpy as np

from .bbox import bbox_from_cells
from .fv import assemble, box_slice
from .krylov import gmres, solve_lu, solve_pcg


def problem_box(prob):
    """The fixed box of a workload, else the cell bounding box with its margin."""
    if prob.box is not None:
        return prob.box
    return bbox_from_cells(prob.cell_id, prob.margin)


def implicit_step(fields, mask, D, k, src, c_b, box, dt, h, solver="auto", tol=1e-13,
                  restart=30):
    """Advance lattice fields ``[S][z][y][x]`` by one step; returns ``(new, infos)``.

    ``solver``: "lu" (dense), "pcg" (Jacobi CG to ``tol``), "gmres" (GMRES(restart)
    to ``tol``) or "auto" (LU up to 512 unknowns, else PCG).  Each species starts
    its iteration from c^n.
    """
    out = np.array(fields, dtype=np.float64, copy=True)
    sl = box_slice(box)
    mb = mask[sl].astype(bool)
    infos = []
    for s in range(fields.shape[0]):
        A, q = assemble(mb, D[s][sl], k[s][sl], src[s][sl], float(c_b[s]), dt, h)
        cn = fields[s][sl][mb]
        b = cn + q
        n = len(b)
        if n == 0:
            infos.append({"n": 0})
            continue
        if solver == "lu" or (solver == "auto" and n <= 512):
            x = solve_lu(A, b)
            info = {"solver": "lu"}
        elif solver in ("pcg", "auto"):
            x, it = solve_pcg(A, b, x0=cn, tol=tol)
            info = {"solver": "pcg", "iterations": it}
        elif solver == "gmres":
            x, info = gmres(A, b, x0=cn, restart=restart, tol=tol)
            info["solver"] = "gmres"
        else:
            raise ValueError(solver)
        info["n"] = n
        info["rel_res"] = float(np.linalg.norm(b - A @ x) / max(np.linalg.norm(b), 1e-300))
        view = out[s][sl]
        view[mb] = x
        infos.append(info)
    return out, infos


def run(prob, steps=None, solver="auto", tol=1e-13, box=None):
    """Run ``steps`` implicit steps of a ``synth.Problem`` on its (fixed) box."""
    box = box if box is not None else problem_box(prob)
    c = prob.c0.copy()
    steps = prob.steps if steps is None else steps
    allinfo = []
    for _ in range(steps):
        c, infos = implicit_step(c, prob.mask, prob.D, prob.k, prob.src, prob.c_b, box,
                                 prob.dt, prob.h, solver=solver, tol=tol)
        allinfo.append(infos)
    return c, allinfo
