"""Krylov invariants of the GPU's delayed classical Gram-Schmidt, checked against the
oracle's own matrix (no GMRES iterate is compared here).

After a step, the basis of the last cycle is read back (``mpm_debug_krylov``): columns
q_1 .. q_{m-1} (q_0 has been overwritten by the next residual at the end of the cycle)
and the unrotated Hessenberg matrix H.  With B = S A S, S = diag(A)^(-1/2), assembled by
the oracle, the Arnoldi relation B q_k = sum_{i <= k+1} H[i][k] q_i gives, for k >= 1,

    w_k = B q_k - sum_{1 <= i <= k+1} H[i][k] q_i = H[0][k] q_0,

so every w_k has norm |H[0][k]|, is orthogonal to q_1 .. q_{m-1}, and all w_k / H[0][k]
are the same unit vector.  The columns q_1 .. q_{m-1} are orthonormal, and since B is
symmetric, H is tridiagonal up to rounding.  Tolerances: the basis is stored in FP32
(inner solve) or FP64, with one reorthogonalisation.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from gpu_helpers import require_gpu, to_dev
from oracle.fv import assemble, box_slice
from synth import random_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [(1, 5e-5), (0, 1e-11)])
@pytest.mark.parametrize("restart", [8, 12])
def test_basis_orthonormal_and_arnoldi_relation(precision, tol, restart):
    torch = require_gpu()
    from paper_2505_03067_amd import Solver
    p = random_problem(72, (22, 21, 19), S=2, fill=0.7)
    box = p.box
    d = to_dev(p)
    f = torch.from_numpy(p.c0).cuda()
    sl = box_slice(box)
    mb = p.mask[sl].astype(bool)
    N = int(mb.sum())
    # one cycle only, to a tolerance it cannot reach: its basis is the one read back
    with Solver(2, 1, precision=precision, restart=restart, max_cycles=1) as s:
        s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        assert s.step([f], 1e-14) == 1        # MPM_NOT_CONVERGED after the single cycle
        for spc in range(2):
            m, vs, V, H = s.krylov(0, spc, restart, N)
            assert m >= 3, m
            A, _ = assemble(mb, p.D[spc][sl], p.k[spc][sl], p.src[spc][sl], float(p.c_b[spc]), p.dt, p.h)
            sc = 1.0 / np.sqrt(A.diagonal())
            B = sp.diags(sc) @ A @ sp.diags(sc)
            Q = vs[:, None] * V                      # rows q_0 .. q_{m-1}; q_0 is stale
            Qr = Q[1:m]
            G = Qr @ Qr.T
            orth = np.abs(G - np.eye(m - 1)).max()
            dirs = []
            for k in range(1, m - 1):
                w = B @ Q[k] - H[k, 1:k + 2] @ Q[1:k + 2]
                h0 = H[k, 0]
                assert abs(np.linalg.norm(w) - abs(h0)) <= tol * max(1.0, abs(h0)) * 10, (k, np.linalg.norm(w), h0)
                assert np.abs(Qr @ w).max() <= tol * 10, k
                if abs(h0) > 1e-3:
                    dirs.append(w / h0)
            for u in dirs[1:]:
                assert np.linalg.norm(u - dirs[0]) <= tol * 100
            print(f"precision {precision} restart {restart} species {spc}: m {m}, "
                  f"orthogonality {orth:.2e}, columns compared {len(dirs)}", flush=True)
            assert orth <= tol, orth
            # the subdiagonal (the norms of the orthogonalised vectors) is positive
            assert all(H[k, k + 1] > 0 for k in range(m - 1))
            # B is symmetric, so H is tridiagonal up to rounding (a Lanczos recurrence)
            far = max((abs(H[k, i]) for k in range(2, m - 1) for i in range(0, k - 1)), default=0.0)
            assert far <= tol * 10, far
