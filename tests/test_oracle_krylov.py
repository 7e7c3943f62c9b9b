"""Pins for the oracle's linear solvers (Sec. 2.4: GMRES of Saad and Schultz)."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.fv import assemble
from oracle.krylov import gmres, solve_lu, solve_pcg
from synth import random_problem


def _system(seed, dims=(7, 6, 5), dt=1.0, h=1.0):
    p = random_problem(seed, dims, S=1, fill=0.65)
    A, q = assemble(p.mask.astype(bool), p.D[0], p.k[0], p.src[0], float(p.c_b[0]), dt, h)
    b = p.c0[0][p.mask.astype(bool)] + q
    return A, b


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_solvers_match_spsolve(seed):
    A, b = _system(seed)
    ref = spla.spsolve(A.tocsc(), b)
    x_lu = solve_lu(A, b)
    x_cg, _ = solve_pcg(A, b, tol=1e-14)
    x_gm, info = gmres(A, b, restart=30, tol=1e-13)
    for x in (x_lu, x_cg, x_gm):
        assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert info["converged"]
    # the reported residual is the true one
    assert abs(info["rel_res"] - np.linalg.norm(b - A @ x_gm) / np.linalg.norm(b)) < 1e-15


def test_gmres_restart_and_history():
    """Short restarts still converge; the in-cycle estimate tracks the true residual."""
    A, b = _system(5, dims=(10, 9, 8), dt=3.0)
    x, info = gmres(A, b, restart=5, tol=1e-10)
    assert info["converged"] and info["cycles"] > 1
    rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert rel <= 1e-10
    # the last estimate of the last cycle is within a small factor of the true residual
    assert info["history"][-1] <= 1e-10 * 1.0001
    assert rel <= 10 * max(info["history"][-1], 1e-16)


def test_gmres_diagonal_distinct_eigenvalues():
    """Without preconditioning, GMRES on a matrix with 3 distinct eigenvalues
    terminates after at most 3 iterations (minimal polynomial of degree 3)."""
    rng = np.random.default_rng(0)
    d = rng.choice([1.0, 2.5, 7.0], size=200)
    A = sp.diags(d).tocsr()
    b = rng.random(200)
    x, info = gmres(A, b, restart=30, tol=1e-12, precondition=False)
    assert info["iterations"] <= 3
    np.testing.assert_allclose(x, b / d, rtol=1e-12)


def test_pcg_zero_rhs_and_warm_start():
    A, b = _system(3)
    x, it = solve_pcg(A, np.zeros_like(b))
    assert it == 0 and not np.any(x)
    exact = solve_lu(A, b)
    x2, it2 = solve_pcg(A, b, x0=exact, tol=1e-12)
    assert it2 <= 1
