"""Growing tumours with a moving bounding box (the paper's box tracking, Sec. 2.3):
several problems of uneven size in one context, the box recomputed on the GPU from
the cell lattice after each growth step, the problems re-set up, and the fields
carried across box changes on the lattice.  Checked against the oracle running the
same sequence."""

import numpy as np
import pytest

from gpu_helpers import rel_err, require_gpu
from oracle.bbox import bbox_from_cells
from oracle.fv import box_slice
from oracle.step import implicit_step
from synth import dilate6, tumour_coefficients
from synth.geometry import _inside_ellipsoid

pytestmark = pytest.mark.gpu


def _tumour(dims, semi):
    mid = tuple(d / 2 for d in dims)
    return _inside_ellipsoid(dims, mid, semi)


@pytest.mark.parametrize("precision", [0, 1])
def test_growing_tumours_track_box(precision):
    torch = require_gpu()
    import paper_2505_03067_amd as m
    lattices = [(36, 34, 30), (28, 30, 26)]
    semis = [(6, 5, 4), (3, 4, 3)]
    rngs = [np.random.default_rng(10 + i) for i in range(2)]
    tumours = [_tumour(d, s) for d, s in zip(lattices, semis)]
    jit = [r.uniform(0.8, 1.2, size=(3,) + t.shape) for r, t in zip(rngs, tumours)]
    cb = np.array([1.0, 1.0, 0.0])
    fields_h = [np.broadcast_to(cb[:, None, None, None], (3,) + t.shape).copy() for t in tumours]
    fields_d = [torch.from_numpy(f).cuda() for f in fields_h]
    masks = [np.ones(t.shape, np.uint8) for t in tumours]
    boxes_seen = []
    with m.Solver(3, 2, precision=precision) as s:
        for step in range(9):
            if step % 3 == 0:
                if step > 0:
                    tumours = [dilate6(t) for t in tumours]
                for p in range(2):
                    cell = tumours[p].astype(np.int32)
                    box = m.mpm_bbox_from_cells(torch.from_numpy(cell).cuda(), 4)
                    assert box == bbox_from_cells(cell, 4)
                    D, k, src = tumour_coefficients(tumours[p], jit[p])
                    s.setup(p, box, torch.from_numpy(masks[p]).cuda(), torch.from_numpy(D).cuda(),
                            torch.from_numpy(k).cuda(), torch.from_numpy(src).cuda(), cb, 1.0, 1.0)
                    boxes_seen.append((p, box))
            s.step(fields_d, 1e-12)
            for p in range(2):
                D, k, src = tumour_coefficients(tumours[p], jit[p])
                box = bbox_from_cells(tumours[p].astype(np.int32), 4)
                fields_h[p], _ = implicit_step(fields_h[p], masks[p], D, k, src, cb, box, 1.0, 1.0,
                                               solver="pcg", tol=1e-13)
    # the boxes grew with the tumours
    assert boxes_seen[0][1] != boxes_seen[-2][1]
    for p in range(2):
        got = fields_d[p].cpu().numpy()
        want = fields_h[p]
        for sp in range(3):
            err = rel_err(got[sp], want[sp])
            assert err <= 1e-8, (p, sp, err)


@pytest.mark.parametrize("precision", [0, 1])
def test_box_shrinks_and_grows_again(precision):
    """One problem re-set up on boxes of changing size: the setup buffers and the Krylov
    workspace are reused when the new box fits (what lies past the new layout is cleared)
    and reallocated when it does not; every step matches the oracle on the same box."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from synth import random_problem
    p = random_problem(61, (40, 36, 30), S=3, fill=0.7)
    boxes = [((0, 0, 0), (40, 36, 30)), ((5, 4, 3), (21, 19, 14)), ((2, 2, 2), (30, 30, 25)),
             ((3, 1, 0), (32, 34, 29)), ((0, 0, 0), (40, 36, 30))]
    d = {k: torch.from_numpy(np.ascontiguousarray(getattr(p, k))).cuda() for k in ("mask", "D", "k", "src")}
    f_d = torch.from_numpy(p.c0).cuda()
    f_h = p.c0.copy()
    with m.Solver(3, 1, precision=precision) as s:
        for box in boxes:
            s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
            s.step([f_d], 1e-12)
            f_h, _ = implicit_step(f_h, p.mask, p.D, p.k, p.src, p.c_b, box, p.dt, p.h,
                                   solver="pcg", tol=1e-13)
            got = f_d.cpu().numpy()
            for sp in range(3):
                err = rel_err(got[sp], f_h[sp])
                assert err <= 1e-8, (box, sp, err)


@pytest.mark.parametrize("precision", [0, 1])
def test_update_coefficients_on_a_standing_box(precision):
    """mpm_fv_update: new D, k and s on the box of the last set-up (the paper re-tracks
    the box only every 50 Monte Carlo steps while the cells change every step).  Each
    step matches the oracle on the same box with the new coefficients, and is
    bit-identical to a context set up afresh with them (same fixed work split)."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from synth import random_problem
    p = random_problem(63, (36, 30, 26), S=3, fill=0.7)
    rng = np.random.default_rng(5)
    box = ((2, 1, 3), (33, 28, 24))
    d = {k: torch.from_numpy(np.ascontiguousarray(getattr(p, k))).cuda() for k in ("mask", "D", "k", "src")}
    f_u = torch.from_numpy(p.c0).cuda()
    f_h = p.c0.copy()
    coefs = [(p.D, p.k, p.src)]
    for _ in range(3):
        D2 = p.D * rng.uniform(0.5, 1.5, size=p.D.shape)
        k2 = p.k * rng.uniform(0.5, 1.5, size=p.k.shape)
        s2 = p.src * rng.uniform(0.5, 1.5, size=p.src.shape)
        coefs.append((D2, k2, s2))
    with m.Solver(3, 1, precision=precision, tile_override=2048) as s:
        for i, (D, k, src) in enumerate(coefs):
            dd = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (D, k, src)]
            f_fresh = f_u.clone()
            if i == 0:
                s.setup(0, box, d["mask"], *dd, p.c_b, p.dt, p.h)
            else:
                s.update(0, d["mask"], *dd, p.c_b, p.dt, p.h)
            s.step([f_u], 1e-12)
            f_h, _ = implicit_step(f_h, p.mask, D, k, src, p.c_b, box, p.dt, p.h, solver="pcg", tol=1e-13)
            got = f_u.cpu().numpy()
            for sp in range(3):
                err = rel_err(got[sp], f_h[sp])
                assert err <= 1e-8, (i, sp, err)
            with m.Solver(3, 1, precision=precision, tile_override=2048) as s2:
                s2.setup(0, box, d["mask"], *dd, p.c_b, p.dt, p.h)
                s2.step([f_fresh], 1e-12)
            assert torch.equal(f_fresh, f_u), i


def test_update_errors():
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from synth import random_problem
    p = random_problem(64, (12, 10, 8), S=3, fill=0.8)
    d = {k: torch.from_numpy(np.ascontiguousarray(getattr(p, k))).cuda() for k in ("mask", "D", "k", "src")}
    with m.Solver(3, 1) as s:
        with pytest.raises(m.MpmError) as e:
            s.update(0, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        assert e.value.code == m.MPM_ESTATE
        s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        with pytest.raises(m.MpmError) as e:
            s.update(0, d["mask"], -d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        assert e.value.code == m.MPM_EINVAL
        with pytest.raises(m.MpmError) as e:
            s.update(0, d["mask"], d["D"], d["k"], d["src"], p.c_b, 0.0, p.h)
        assert e.value.code == m.MPM_EINVAL
