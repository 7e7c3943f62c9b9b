"""Pins for the oracle's finite-volume step (Sec. 2.2 eqs. 1-4, Sec. 2.4).

Nothing here re-types the oracle's formulas: each test checks an independent fact
(hand-derived fixtures, closed-form Fourier decay, conservation, maximum principle,
analytic steady profiles, matrix structure).
"""

from fractions import Fraction

import numpy as np
import pytest

from conftest import parse_cases
from oracle.fv import assemble, harmonic_mean
from oracle.step import implicit_step
from synth import fourier_box, random_problem


def _frac_list(tokens):
    return [Fraction(t) for t in tokens]


@pytest.mark.parametrize("case", parse_cases("fv_cases.txt"), ids=lambda c: c["name"])
def test_hand_derived_cases(case):
    nx, ny, nz = (int(v) for v in case["dims"])
    shape = (1, nz, ny, nx)
    arr = lambda key: np.array([float(v) for v in _frac_list(case[key])]).reshape(shape)
    mask = np.array([int(v) for v in case["mask"]], np.uint8).reshape(shape[1:])
    cn = arr("cn")
    out, _ = implicit_step(cn, mask, arr("D"), arr("k"), arr("s"),
                           np.array([float(Fraction(case["cb"][0]))]), ((0, 0, 0), (nx, ny, nz)),
                           float(Fraction(case["dt"][0])), float(Fraction(case["h"][0])),
                           solver="lu")
    got_in = out[0][mask.astype(bool)]
    got_out = out[0][~mask.astype(bool)]
    want_in = np.array([float(v) for v in _frac_list(case["expect"])])
    want_out = np.array([float(v) for v in _frac_list(case["keep"])])
    np.testing.assert_allclose(got_in, want_in, rtol=1e-14, atol=0)
    np.testing.assert_array_equal(got_out, want_out)


def _dst_mode(dims, modes):
    """prod_d sin(pi m_d (i_d + 1/2) / N_d) as a [z][y][x] array."""
    axes = []
    for n, m in zip(dims, modes):
        i = np.arange(n)
        axes.append(np.sin(np.pi * m * (i + 0.5) / n))
    x, y, z = axes
    return z[:, None, None] * y[None, :, None] * x[None, None, :]


def _dct_mode(dims, modes):
    axes = []
    for n, m in zip(dims, modes):
        i = np.arange(n)
        axes.append(np.cos(np.pi * m * (i + 0.5) / n))
    x, y, z = axes
    return z[:, None, None] * y[None, :, None] * x[None, None, :]


def _lam(dims, modes, h):
    return sum(4.0 / h ** 2 * np.sin(np.pi * m / (2.0 * n)) ** 2 for n, m in zip(dims, modes))


@pytest.mark.parametrize("dims,modes,D,k,dt,h,cb", [
    ((6, 5, 4), (1, 1, 1), 1.0, 0.0, 1.0, 1.0, 1.0),
    ((6, 5, 4), (3, 2, 4), 0.7, 0.0, 0.5, 1.0, 0.3),
    ((7, 4, 5), (7, 1, 2), 1.3, 0.2, 1.0, 2.0, 0.0),
    ((8, 8, 8), (2, 5, 8), 0.3, 0.05, 2.0, 0.5, 0.0),
])
def test_fourier_decay_dirichlet(dims, modes, D, k, dt, h, cb):
    """Half-cell Dirichlet faces make the DST-II modes exact eigenvectors of the step."""
    p = fourier_box(dims, D=D, k=k, c_b=cb)
    A0 = 0.25
    c0 = (cb + A0 * _dst_mode(dims, modes))[None]
    out, _ = implicit_step(c0, p.mask, p.D, p.k, p.src, p.c_b, p.box, dt, h, solver="lu")
    g = 1.0 / (1.0 + dt * (k + D * _lam(dims, modes, h)))
    np.testing.assert_allclose(out[0] - cb, g * (c0[0] - cb), rtol=0, atol=1e-14)


@pytest.mark.parametrize("dims,modes,D,k,dt,h", [
    ((8, 7, 6), (0, 0, 0), 1.0, 0.0, 1.0, 1.0),
    ((8, 7, 6), (1, 2, 3), 0.9, 0.0, 1.0, 1.0),
    ((9, 6, 7), (5, 0, 2), 0.4, 0.1, 0.7, 1.5, ),
])
def test_fourier_decay_zero_flux(dims, modes, D, k, dt, h):
    """With the domain shrunk away from the box faces, DCT-II modes decay exactly."""
    p = fourier_box(dims, D=D, k=k, c_b=5.0, interior_only=True)
    inner = tuple(n - 2 for n in dims)
    mode = _dct_mode(inner, modes)
    c0 = np.full((1,) + dims[::-1], 2.0)
    c0[0, 1:-1, 1:-1, 1:-1] = 0.5 + 0.25 * mode
    out, _ = implicit_step(c0, p.mask, p.D, p.k, p.src, p.c_b, p.box, dt, h, solver="lu")
    g = 1.0 / (1.0 + dt * (k + D * _lam(inner, modes, h)))
    got = out[0, 1:-1, 1:-1, 1:-1]
    # the constant part decays with 1/(1 + dt k) only
    want = 0.5 / (1.0 + dt * k) + g * 0.25 * mode
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
    # voxels outside the mask are never written
    assert np.all(out[0][p.mask == 0] == 2.0)


def _interior_random(seed, dims, S=2):
    p = random_problem(seed, dims, S=S, fill=0.7)
    p.mask[[0, -1], :, :] = 0
    p.mask[:, [0, -1], :] = 0
    p.mask[:, :, [0, -1]] = 0
    return p


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mass_conservation_zero_flux(seed):
    """No Dirichlet face and k = 0: total mass grows by exactly dt * sum(s)."""
    p = _interior_random(seed, (9, 8, 7))
    p.k[:] = 0.0
    out, _ = implicit_step(p.c0, p.mask, p.D, p.k, p.src, p.c_b, p.box, 0.8, 1.0, solver="lu")
    m = p.mask.astype(bool)
    for s in range(p.nspecies):
        before = p.c0[s][m].sum() + 0.8 * p.src[s][m].sum()
        assert abs(out[s][m].sum() - before) <= 1e-12 * abs(before)


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_maximum_principle(seed):
    """M-matrix: with s = 0 the new field stays within the old values and c_b."""
    p = random_problem(seed, (8, 9, 7), S=2, fill=0.6)
    p.src[:] = 0.0
    m = p.mask.astype(bool)
    out, _ = implicit_step(p.c0, p.mask, p.D, p.k, p.src, p.c_b, p.box, 1.0, 1.0, solver="lu")
    for s in range(p.nspecies):
        hi = max(p.c0[s][m].max(), p.c_b[s])
        assert out[s][m].min() >= -1e-15
        assert out[s][m].max() <= hi + 1e-14
    p.k[:] = 0.0
    out, _ = implicit_step(p.c0, p.mask, p.D, p.k, p.src, p.c_b, p.box, 1.0, 1.0, solver="lu")
    for s in range(p.nspecies):
        lo = min(p.c0[s][m].min(), p.c_b[s])
        hi = max(p.c0[s][m].max(), p.c_b[s])
        assert out[s][m].min() >= lo - 1e-14
        assert out[s][m].max() <= hi + 1e-14


def test_constant_state():
    """k = s = 0 and c^n = c_b everywhere: the step returns c_b."""
    p = random_problem(7, (7, 6, 9), S=3)
    p.k[:] = 0.0
    p.src[:] = 0.0
    c0 = np.broadcast_to(p.c_b[:, None, None, None], p.c0.shape).copy()
    out, _ = implicit_step(c0, p.mask, p.D, p.k, p.src, p.c_b, p.box, 1.0, 1.0, solver="lu")
    np.testing.assert_allclose(out, c0, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("D1,D2,m", [(1.0, 0.25, 5), (0.3, 2.0, 3), (1.0, 1.0, 4)])
def test_two_material_slab_steady_profile(D1, D2, m):
    """Piecewise-linear steady profile across a material interface is a fixed point.

    One active row (x = 1..nx-1) of a 3-voxel-thick box: its y/z faces see voxels
    outside the mask (no flux), x = 0 is outside the mask (closed end), the right end
    is a Dirichlet box face.  All production sits in voxel 1, so the flux F = s h is
    constant from the centre of voxel 1 to the right face, and the exact continuous
    profile is c(x) = c_b + F * integral_x^L dxi / D(xi).  Only the harmonic-mean face
    diffusivity reproduces it at the voxel centres.
    """
    nx, h, s1, cb = 10, 1.0, 0.2, 0.5
    L = nx * h
    xs = (np.arange(nx) + 0.5) * h
    iface = m * h                          # interface between voxels m-1 and m
    F = s1 * h

    def integral(x):                       # integral_x^L dxi / D(xi)
        if x >= iface:
            return (L - x) / D2
        return (iface - x) / D1 + (L - iface) / D2

    prof = np.array([cb + F * integral(x) for x in xs])
    dims = (nx, 3, 3)
    mask = np.zeros((3, 3, nx), np.uint8)
    mask[1, 1, 1:] = 1
    D = np.where(np.arange(nx) < m, D1, D2) * np.ones((1, 3, 3, nx))
    k = np.zeros_like(D)
    src = np.zeros_like(D)
    src[0, 1, 1, 1] = s1
    c0 = np.zeros_like(D)
    c0[0, 1, 1, :] = prof
    out, _ = implicit_step(c0, mask, D, k, src, np.array([cb]), ((0, 0, 0), dims), 1.0, h,
                           solver="lu")
    np.testing.assert_allclose(out[0, 1, 1, 1:], prof[1:], rtol=0, atol=1e-13)


def test_operator_structure():
    """A is symmetric, has positive diagonal, non-positive off-diagonal, and is
    diagonally dominant (an M-matrix); harmonic_mean handles the zero/zero face."""
    p = random_problem(11, (6, 7, 5), S=1, fill=0.7)
    A, _ = assemble(p.mask.astype(bool), p.D[0], p.k[0], p.src[0], 1.0, 0.9, 1.1)
    Ad = A.toarray()
    np.testing.assert_allclose(Ad, Ad.T, rtol=0, atol=0)
    off = Ad - np.diag(np.diag(Ad))
    assert np.all(off <= 0)
    assert np.all(np.diag(Ad) > 0)
    assert np.all(np.diag(Ad) + off.sum(axis=1) >= 1.0 - 1e-14)
    assert harmonic_mean(np.array([0.0]), np.array([0.0]))[0] == 0.0
    assert harmonic_mean(np.array([2.0]), np.array([0.0]))[0] == 0.0
