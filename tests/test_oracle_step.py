"""Whole-step pins for the oracle (Sec. 2.3-2.4)."""

import numpy as np
import pytest

from oracle.step import implicit_step, run
from synth import config1, random_problem


def test_config1_symmetry_and_solver_agreement():
    """config1 is mirror- and permutation-symmetric; LU-free solvers agree."""
    p = config1()
    c_cg, _ = run(p, steps=3, solver="pcg", tol=1e-13)
    c_gm, infos = run(p, steps=3, solver="gmres", tol=1e-12)
    f = c_cg[0]
    np.testing.assert_allclose(f, f[::-1, :, :], atol=1e-12)
    np.testing.assert_allclose(f, f[:, ::-1, :], atol=1e-12)
    np.testing.assert_allclose(f, f[:, :, ::-1], atol=1e-12)
    np.testing.assert_allclose(f, np.transpose(f, (1, 0, 2)), atol=1e-12)
    np.testing.assert_allclose(f, np.transpose(f, (2, 1, 0)), atol=1e-12)
    assert np.linalg.norm(c_cg - c_gm) <= 1e-10 * np.linalg.norm(c_cg)
    assert 0.0 < f.min() < 1.0 and f.max() <= 1.0 + 1e-14
    # GMRES(30) + Jacobi needs a few tens of iterations per step on this problem
    its = [i[0]["iterations"] for i in infos]
    assert all(15 <= it <= 60 for it in its)


@pytest.mark.slow
def test_config1_ten_steps_minimum():
    p = config1()
    c, _ = run(p, solver="pcg", tol=1e-13)
    assert 0.39 < c.min() < 0.41


def test_box_restriction_leaves_outside_untouched():
    p = random_problem(21, (10, 9, 8), S=2)
    box = ((2, 1, 3), (8, 7, 6))
    out, _ = implicit_step(p.c0, p.mask, p.D, p.k, p.src, p.c_b, box, 1.0, 1.0, solver="lu")
    inside = np.zeros(p.mask.shape, bool)
    inside[3:6, 1:7, 2:8] = True
    touched = inside & p.mask.astype(bool)
    assert np.array_equal(out[:, ~touched], p.c0[:, ~touched])
    assert np.any(out[:, touched] != p.c0[:, touched])


def test_species_independence():
    """Identical species coefficients give identical fields (no cross-coupling)."""
    p = random_problem(22, (7, 7, 7), S=3)
    for a in (p.D, p.k, p.src, p.c0):
        a[1] = a[0]
        a[2] = a[0]
    p.c_b[1] = p.c_b[2] = p.c_b[0]
    out, _ = implicit_step(p.c0, p.mask, p.D, p.k, p.src, p.c_b, p.box, 1.0, 1.0, solver="pcg")
    np.testing.assert_array_equal(out[0], out[1])
    np.testing.assert_array_equal(out[0], out[2])
