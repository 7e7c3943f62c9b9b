"""Linear solvers for the per-step system A c^{n+1} = b (Sec. 2.4).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper solves each implicit step with GMRES (Saad and Schultz) through
PETSc.  It states no restart length, preconditioner or tolerance; the readings
used here are GMRES(30) with Jacobi preconditioning and a relative residual
||b - A x||_2 / ||b||_2 measured in FP64.

Three solvers, all FP64:

* ``solve_lu``   - dense LU through LAPACK (small boxes), the exact answer;
* ``solve_pcg``  - Jacobi-preconditioned conjugate gradients; A is symmetric
                   positive definite, so this converges to the same unique
                   solution and is the parity reference for larger boxes;
* ``gmres``      - restarted GMRES(m) with modified Gram-Schmidt Arnoldi,
                   right Jacobi preconditioning and Givens rotations; used to
                   time the method as the paper runs it and for iteration-count
                   context.

Pinned by (``tests/test_oracle_krylov.py``): agreement of all three with
``scipy.sparse.linalg.spsolve`` on random SPD M-matrices from the assembly,
the residual each one reports recomputed independently, GMRES on a diagonal
matrix (converges in as many iterations as distinct eigenvalues), and the
Givens residual estimate matching the true residual.
"""

from __future__ import annotations

import numpy as np


def solve_lu(A, b):
    """Exact solve by dense LU (numpy.linalg.solve)."""
    return np.linalg.solve(A.toarray(), b)


def solve_pcg(A, b, x0=None, tol=1e-13, maxiter=100000):
    """Jacobi-preconditioned CG to ||b - A x|| <= tol ||b||; returns (x, iterations).

    Standard preconditioned CG: r = b - A x, z = M^{-1} r, p = z, then per iteration
    alpha = (r.z)/(p.Ap), x += alpha p, r -= alpha Ap, z = M^{-1} r,
    beta = (r_new.z_new)/(r.z), p = z + beta p.  The final residual is recomputed.
    """
    n = A.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0
    dinv = 1.0 / A.diagonal()
    r = b - A @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * bnorm and it < maxiter:
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    r = b - A @ x
    if np.linalg.norm(r) > tol * bnorm * 10.0:
        raise RuntimeError("PCG did not reach the requested residual")
    return x, it


def gmres(A, b, x0=None, restart=30, tol=1e-8, max_cycles=200, precondition=True):
    """Restarted GMRES(m), modified Gram-Schmidt, right Jacobi preconditioning.

    Stops when the true FP64 residual ||b - A x|| is at most tol ||b||; that test is
    made at the end of every cycle on the recomputed residual, and inside a cycle
    the Givens estimate decides when to close the cycle early.

    Returns ``(x, info)`` with ``info = {"iterations", "cycles", "history",
    "converged", "rel_res"}``; ``history`` holds the in-cycle residual estimates.
    """
    n = A.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    info = {"iterations": 0, "cycles": 0, "history": [], "converged": False}
    if bnorm == 0.0:
        info.update(converged=True, rel_res=0.0)
        return np.zeros(n), info
    minv = 1.0 / A.diagonal() if precondition else np.ones(n)
    m = restart
    for _ in range(max_cycles):
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            info.update(converged=True, rel_res=beta / bnorm)
            return x, info
        info["cycles"] += 1
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(m):
            w = A @ (minv * V[j])                       # A M^{-1} v_j
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = w @ V[i]
                w -= H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                          # previous rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = np.hypot(H[j, j], H[j + 1, j])         # new rotation zeroes H[j+1, j]
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k_used = j + 1
            info["iterations"] += 1
            info["history"].append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm:
                break
        y = np.zeros(k_used)                            # back-substitution R y = g
        for i in range(k_used - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k_used] @ y[i + 1:]) / H[i, i]
        x = x + minv * (y @ V[:k_used])
    r = b - A @ x
    rel = np.linalg.norm(r) / bnorm
    info.update(converged=bool(rel <= tol), rel_res=rel)
    return x, info
