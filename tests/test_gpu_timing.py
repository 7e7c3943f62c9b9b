"""The kernel-timing hook: counts launches and bytes, and does not change results."""

import numpy as np
import pytest

from gpu_helpers import rel_err, require_gpu, to_dev
from synth import random_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("opts", [dict(), dict(use_graph=1), dict(batched=0), dict(ortho=0),
                                  dict(ortho=0, batched=0)])
@pytest.mark.parametrize("kind,j", [(2, 3), (1, 0), (3, 5), (4, 0), (5, 0)])
def test_timing_hook(opts, kind, j):
    torch = require_gpu()
    from paper_2505_03067_amd import MPM_ORTHO_DCGS2, MpmError, Solver
    if kind == 3 and opts.get("ortho", MPM_ORTHO_DCGS2) == MPM_ORTHO_DCGS2:
        # the delayed scheme has no separate axpy+norm kernel: refused
        with Solver(3, 1) as s:
            with pytest.raises(MpmError):
                s.time_kernel(kind, j)
        return
    p = random_problem(71, (30, 27, 25), S=3, fill=0.6)
    d = to_dev(p)
    res = []
    for timed in (False, True):
        f = torch.from_numpy(p.c0).cuda()
        with Solver(3, 1, tile_override=1024, **opts) as s:
            s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, 1.0, 1.0)
            if timed:
                s.time_kernel(kind, j)
            for _ in range(2):
                s.step([f], 1e-10)
            t = s.kernel_timing()
            cyc = sum(s.stats(0, sp)["cycles"] for sp in range(3))
        res.append(f.cpu().numpy())
        if timed:
            assert t["launches"] >= 2 and t["ms"] > 0 and t["bytes"] > 0, t
        else:
            assert t["launches"] == 0
    assert np.array_equal(res[0], res[1])
    assert cyc >= 1


def test_autotuned_split_is_reported_and_parity_holds():
    torch = require_gpu()
    from paper_2505_03067_amd import Solver
    from oracle.fv import box_slice
    from oracle.step import run
    p = random_problem(72, (40, 36, 30), S=3, fill=0.7)
    d = to_dev(p)
    f = torch.from_numpy(p.c0).cuda()
    with Solver(3, 1) as s:
        s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, 1.0, 1.0)
        s.step([f], 1e-12)
        tile = s.tile()
    assert tile >= 1024 and tile % 1024 == 0
    want, _ = run(p, steps=1, solver="pcg", tol=1e-13)
    mb = p.mask.astype(bool)
    got = f.cpu().numpy()
    for sp in range(3):
        err = rel_err(got[sp][mb], want[sp][mb])
        assert err <= 1e-8


@pytest.mark.parametrize("kind,j", [(1, 4), (5, 0)])
def test_timing_repeat_leaves_results_unchanged(kind, j):
    """Repeated back-to-back launches of a kernel whose output depends on its inputs
    alone change nothing; the launch count includes every repeat."""
    torch = require_gpu()
    from paper_2505_03067_amd import MpmError, Solver
    p = random_problem(73, (28, 26, 24), S=3, fill=0.6)
    d = to_dev(p)
    res, counts = [], []
    for rep in (0, 1, 7):
        f = torch.from_numpy(p.c0).cuda()
        with Solver(3, 1, tile_override=1024) as s:
            s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, 1.0, 1.0)
            if rep:
                s.time_kernel(kind, j, rep)
            for _ in range(2):
                s.step([f], 1e-10)
            counts.append(s.kernel_timing()["launches"])
            if rep == 7:
                with pytest.raises(MpmError):
                    s.time_kernel(2, j, 2)          # the axpy kernel updates its input in place
        res.append(f.cpu().numpy())
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])
    assert counts[0] == 0 and counts[1] >= 1 and counts[2] == 7 * counts[1]
