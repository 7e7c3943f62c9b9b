"""Shared helpers for the GPU tests: run the HIP path and the oracle on one input.

The two sides share only the generator's arrays; the oracle never sees anything the
GPU produced except for the final comparison.
"""

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    import paper_2505_03067_amd as m
    m.lib()          # raises ImportError if libmpm.so is missing: never silently skipped
    return torch


def to_dev(prob):
    import torch
    dev = torch.device("cuda")
    return dict(mask=torch.from_numpy(np.ascontiguousarray(prob.mask)).to(dev),
                D=torch.from_numpy(np.ascontiguousarray(prob.D)).to(dev),
                k=torch.from_numpy(np.ascontiguousarray(prob.k)).to(dev),
                src=torch.from_numpy(np.ascontiguousarray(prob.src)).to(dev))


def gpu_run(prob, steps, tol, box=None, c0=None, **opts):
    """Run ``steps`` GPU steps of one problem; returns (fields, [stats per step])."""
    import torch
    from paper_2505_03067_amd import Solver
    from oracle.step import problem_box  # box choice only (the oracle's bbox is pinned)
    box = box if box is not None else problem_box(prob)
    d = to_dev(prob)
    f = torch.from_numpy(np.ascontiguousarray(prob.c0 if c0 is None else c0)).cuda()
    stats = []
    with Solver(prob.nspecies, 1, **opts) as s:
        s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], prob.c_b, prob.dt, prob.h)
        for _ in range(steps):
            s.step([f], tol)
            stats.append([s.stats(0, sp) for sp in range(prob.nspecies)])
    torch.cuda.synchronize()
    return f.cpu().numpy(), stats


def err_norms(got, want, mask_box_bool, box):
    """Per species, over the domain voxels of the box: (relative L2 error
    ||g - w||_2 / ||w||_2, relative max-norm error max|g - w| / max|w|)."""
    from oracle.fv import box_slice
    sl = box_slice(box)
    out = []
    for s in range(got.shape[0]):
        g = got[s][sl][mask_box_bool]
        w = want[s][sl][mask_box_bool]
        l2 = float(np.linalg.norm(g - w) / max(np.linalg.norm(w), 1e-300))
        mx = float(np.max(np.abs(g - w)) / max(np.max(np.abs(w)), 1e-300)) if g.size else 0.0
        out.append((l2, mx))
    return out


def rel_err(g, w):
    """The larger of the relative L2 and relative max-norm errors of two arrays."""
    g = np.asarray(g).ravel()
    w = np.asarray(w).ravel()
    l2 = float(np.linalg.norm(g - w) / max(np.linalg.norm(w), 1e-300))
    mx = float(np.max(np.abs(g - w)) / max(np.max(np.abs(w)), 1e-300)) if g.size else 0.0
    return max(l2, mx)


def rel_err_per_species(got, want, mask_box_bool, box):
    """Per species, the larger of the relative L2 and relative max-norm errors (both must
    meet a parity bar, so a single voxel far off cannot hide in the L2 norm)."""
    return [max(l2, mx) for l2, mx in err_norms(got, want, mask_box_bool, box)]
