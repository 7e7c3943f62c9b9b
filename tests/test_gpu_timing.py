"""The kernel-timing hook: counts launches and bytes, and does not change results."""

import numpy as np
import pytest

from gpu_helpers import require_gpu, to_dev
from synth import random_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("opts", [dict(), dict(use_graph=0), dict(batched=0)])
@pytest.mark.parametrize("kind,j", [(2, 3), (1, 0), (3, 5), (4, 0), (5, 0)])
def test_timing_hook(opts, kind, j):
    torch = require_gpu()
    from paper_2505_03067_amd import Solver
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
        err = np.linalg.norm(got[sp][mb] - want[sp][mb]) / np.linalg.norm(want[sp][mb])
        assert err <= 1e-8
