"""Parity at the benchmark sizes, in the launch configuration bench.py times (batched,
FP32 GMRES(30) in FP64 refinement, delayed CGS2, direct launches, autotuned split).

* Config 2 (128^3 box of the 256x256x160 lattice, 709,620 unknowns): every field
  against the oracle's CG solve, 1e-8 relative per species, as the small cases.
* Config 5 (384x384x256 box of the 512x512x320 lattice, 6.4 M unknowns) with cell
  growth between steps: the box recomputed on the GPU is bit-exact against the
  oracle's brute force, and the relative FP64 residual of each returned field,
  recomputed from the oracle's own assembly, meets the tolerance (a property that holds
  at any size; a full CG solve of 6.4 M unknowns per step is too slow for a test).
  Voxels outside the box or the domain come back bit-identical.
"""

import numpy as np
import pytest

from gpu_helpers import rel_err_per_species, require_gpu, to_dev
from oracle.bbox import bbox_from_cells
from oracle.fv import assemble, box_slice
from oracle.step import run

pytestmark = pytest.mark.gpu


def test_config2_full_size_parity():
    torch = require_gpu()
    from paper_2505_03067_amd import Solver
    from synth import config2
    p = config2()
    box = bbox_from_cells(p.cell_id, p.margin)
    d = to_dev(p)
    f = torch.from_numpy(p.c0).cuda()
    steps = 3
    with Solver(3, 1) as s:
        s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        for _ in range(steps):
            s.step([f], 1e-12)
        stats = [s.stats(0, sp) for sp in range(3)]
    got = f.cpu().numpy()
    want, _ = run(p, steps=steps, solver="pcg", tol=1e-13, box=box)
    mb = p.mask[box_slice(box)].astype(bool)
    errs = rel_err_per_species(got, want, mb, box)
    print(f"config2 full size: rel_err {errs}, iterations {[st['iterations'] for st in stats]}", flush=True)
    assert max(errs) <= 1e-8, errs
    touched = np.zeros(p.mask.shape, bool)
    touched[box_slice(box)] = mb
    assert np.array_equal(got[:, ~touched], p.c0[:, ~touched])


def test_config5_full_size_with_growth():
    torch = require_gpu()
    from paper_2505_03067_amd import Solver, mpm_bbox_from_cells
    from synth import config5
    from synth.geometry import grow_cells
    p = config5()
    tol = 1e-8
    growth = grow_cells(p, 2)
    cell = p.cell_id.copy()
    k, src = p.k.copy(), p.src.copy()
    d = to_dev(p)
    cell_d = torch.from_numpy(cell).cuda()
    f = torch.from_numpy(p.c0).cuda()
    S = p.nspecies
    prev = p.c0.copy()
    with Solver(S, 1) as s:
        for g in growth:
            # the same growth on both sides
            flat = cell.reshape(-1)
            flat[g.index] = g.cell
            k.reshape(S, -1)[:, g.index] = g.k
            src.reshape(S, -1)[:, g.index] = g.src
            idx = torch.from_numpy(g.index).cuda()
            cell_d.view(-1)[idx] = torch.from_numpy(g.cell).cuda()
            d["k"].view(S, -1)[:, idx] = torch.from_numpy(g.k).cuda()
            d["src"].view(S, -1)[:, idx] = torch.from_numpy(g.src).cuda()
            box = mpm_bbox_from_cells(cell_d, p.margin)
            assert box == bbox_from_cells(cell, p.margin)
            s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
            s.step([f], tol)
            got = f.cpu().numpy()
            sl = box_slice(box)
            mb = p.mask[sl].astype(bool)
            for sp in range(S):
                A, q = assemble(mb, p.D[sp][sl], k[sp][sl], src[sp][sl], float(p.c_b[sp]), p.dt, p.h)
                b = prev[sp][sl][mb] + q
                r = b - A @ got[sp][sl][mb]
                rel = np.linalg.norm(r) / np.linalg.norm(b)
                print(f"config5 box {box} species {sp}: oracle residual {rel:.3e}", flush=True)
                assert rel <= tol * (1 + 1e-6), (sp, rel)
            touched = np.zeros(p.mask.shape, bool)
            touched[sl] = mb
            assert np.array_equal(got[:, ~touched], prev[:, ~touched])
            prev = got
