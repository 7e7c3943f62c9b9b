"""Pins for the FP64 U-Net oracle (brute force, identities, finite differences)."""

import numpy as np
import pytest

from oracle import unet


def test_parameter_count_of_the_specified_network():
    assert unet.param_count(13, 3, [16, 32, 64, 64]) == 911715


def test_conv3_matches_brute_force_loop():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(1, 3, 4, 5, 2))
    W = rng.normal(size=(27, 2, 3))
    b = rng.normal(size=3)
    got = unet.conv3(x, W, b)
    n, D, H, Wd, ci = x.shape
    for z in range(D):
        for y in range(H):
            for xx in range(Wd):
                for co in range(3):
                    acc = b[co]
                    for kz in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                zz, yy, x2 = z + kz - 1, y + ky - 1, xx + kx - 1
                                if 0 <= zz < D and 0 <= yy < H and 0 <= x2 < Wd:
                                    t = kz * 9 + ky * 3 + kx
                                    for c in range(ci):
                                        acc += x[0, zz, yy, x2, c] * W[t, c, co]
                    assert abs(got[0, z, y, xx, co] - acc) < 1e-12


def test_conv3_delta_kernel_is_identity_and_shift():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 4, 4, 4, 3))
    W = np.zeros((27, 3, 3))
    W[13] = np.eye(3)                                # centre tap
    np.testing.assert_allclose(unet.conv3(x, W, np.zeros(3)), x, atol=0)
    W = np.zeros((27, 3, 3))
    W[14] = np.eye(3)                                # dx = +1: out[x] = in[x + 1]
    out = unet.conv3(x, W, np.zeros(3))
    np.testing.assert_allclose(out[:, :, :, :-1], x[:, :, :, 1:], atol=0)
    assert np.all(out[:, :, :, -1] == 0)


def test_pool_and_upsample_identities():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 4, 6, 2, 3))
    np.testing.assert_allclose(unet.pool2(unet.up2(x)), x, atol=1e-15)
    c = np.full((1, 4, 4, 4, 2), 3.5)
    np.testing.assert_allclose(unet.pool2(c), 3.5)


@pytest.mark.parametrize("widths", [[2, 3], [2, 3, 4, 4]])
def test_gradients_match_central_differences(widths):
    rng = np.random.default_rng(3)
    in_ch, out_ch = 3, 2
    P = unet.param_count(in_ch, out_ch, widths)
    theta = rng.normal(scale=0.4, size=P)
    # shift the biases up so that ReLUs are mostly active but some are not
    x = rng.normal(size=(1, 8, 8, 8, in_ch))
    target = rng.normal(size=(1, 8, 8, 8, out_ch))

    def loss(th):
        return unet.mse(unet.forward(th, x, in_ch, out_ch, widths), target)[0]

    out, acts = unet.forward(theta, x, in_ch, out_ch, widths, keep=True)
    _, dout = unet.mse(out, target)
    g, dx = unet.backward(theta, acts, dout, in_ch, out_ch, widths)
    assert g.shape == theta.shape
    idx = rng.choice(P, size=40, replace=False)
    eps = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        fd = (loss(tp) - loss(tm)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])
    # gradient with respect to the input as well
    for (n, z, y, xx, c) in [(0, 1, 2, 3, 0), (0, 7, 0, 4, 2), (0, 4, 4, 4, 1)]:
        xp = x.copy(); xp[n, z, y, xx, c] += eps
        xm = x.copy(); xm[n, z, y, xx, c] -= eps
        fd = (unet.mse(unet.forward(theta, xp, in_ch, out_ch, widths), target)[0] -
              unet.mse(unet.forward(theta, xm, in_ch, out_ch, widths), target)[0]) / (2 * eps)
        assert abs(fd - dx[n, z, y, xx, c]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    new = unet.adam(th.copy(), g, m, v, 1, lr=1e-2, eps=0.0)
    np.testing.assert_allclose(new - th, -1e-2 * np.sign(g), rtol=1e-12)
