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


def _torch_bf16(a):
    """PyTorch's CPU float32 -> bfloat16 cast, widened back: an implementation of the
    rounding independent of the oracle's."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32)))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def _same(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    both_nan = np.isnan(a) & np.isnan(b)
    return np.all(both_nan | (a == b)) and np.array_equal(np.signbit(a) | both_nan, np.signbit(b) | both_nan)


def test_bf16_matches_torch_cast_on_edge_cases():
    """Round to nearest with ties to even, signed zeros, the subnormals, overflow to
    infinity, +-Inf and NaN (whatever its payload or sign) against PyTorch's cast."""
    bits = []
    for hi in (0x0000, 0x0001, 0x007F, 0x0080, 0x3F80, 0x3F81, 0x4049, 0x7F7F, 0x7F80, 0x7FC0,
               0x8000, 0x8001, 0x807F, 0xBF80, 0xFF7F, 0xFF80, 0xFFC0, 0x7F81, 0xFFFF):
        for lo in (0x0000, 0x0001, 0x7FFF, 0x8000, 0x8001, 0xFFFF):
            bits.append((hi << 16) | lo)
    a = np.array(bits, dtype=np.uint32).view(np.float32)
    got = unet.bf16(a)
    want = _torch_bf16(a)
    assert _same(got, want)
    # ties: exactly half-way between two BF16 values round to the even one
    one = np.float32(1.0)
    half_ulp = np.float32(2.0 ** -8)
    assert unet.bf16(one + half_ulp) == 1.0                       # tie, 1.0 is even
    assert unet.bf16(np.float32(1.0 + 2.0 ** -7 + 2.0 ** -8)) == 1.0 + 2.0 ** -6   # tie to even above
    big = np.array([0x7F7F7FFF, 0x7F7F8000], np.uint32).view(np.float32)
    assert unet.bf16(big[0]) == np.array(0x7F7F0000, np.uint32).view(np.float32)   # largest BF16
    assert np.isinf(unet.bf16(big[1]))                        # the tie above it rounds to even: Inf
    assert np.isnan(unet.bf16(np.array([0x7FFFFFFF, 0xFFFFFFFF], np.uint32).view(np.float32))).all()


def test_bf16_matches_torch_cast_on_random_bit_patterns():
    rng = np.random.default_rng(11)
    u = rng.integers(0, 2 ** 32, size=200_000, dtype=np.uint64).astype(np.uint32)
    a = u.view(np.float32)
    assert _same(unet.bf16(a), _torch_bf16(a))
    # and on ordinary FP64 data (rounded to FP32 first, as the GPU stores FP32 sums)
    x = rng.normal(scale=3.0, size=100_000) * 10.0 ** rng.integers(-30, 30, size=100_000)
    assert _same(unet.bf16(x), _torch_bf16(x.astype(np.float32)))


def _bf16_exact(a):
    return _same(a, _torch_bf16(a))


def test_store_bf16_rounds_at_every_stored_tensor(monkeypatch):
    """With store_bf16=True the oracle rounds exactly where the GPU stores BF16: the
    3x3x3 weights, every convolution input and output (pooled tensors, concatenations of
    stored tensors) and, in the backward pass, every gradient a convolution reads and the
    input gradient it produces; the head and every bias stay FP32/FP64.  Checked by
    recording what the convolutions see and testing each array against PyTorch's cast;
    with store_bf16=False the same arrays are not BF16 values."""
    rng = np.random.default_rng(12)
    in_ch, out_ch, widths = 3, 2, [2, 3, 4]
    P = unet.param_count(in_ch, out_ch, widths)
    theta = rng.normal(scale=0.5, size=P)
    for W, b in unet.unpack(theta, in_ch, out_ch, widths):
        b[:] = np.abs(b) * 0.1
    x = _torch_bf16(rng.normal(size=(1, 8, 8, 8, in_ch)))
    target = rng.normal(size=(1, 8, 8, 8, out_ch))
    seen = {"fwd": [], "bwd": []}
    c3, c3b = unet.conv3, unet.conv3_backward

    def rec_conv3(a, W, b):
        y = c3(a, W, b)
        seen["fwd"].append((a, W))
        return y

    def rec_conv3_backward(a, W, dy):
        dx, dW, db = c3b(a, W, dy)
        seen["bwd"].append((a, W, dy))
        return dx, dW, db

    monkeypatch.setattr(unet, "conv3", rec_conv3)
    monkeypatch.setattr(unet, "conv3_backward", rec_conv3_backward)
    for store in (True, False):
        seen["fwd"].clear()
        seen["bwd"].clear()
        out, acts = unet.forward(theta, x, in_ch, out_ch, widths, keep=True, store_bf16=store)
        _, dout = unet.mse(out, target)
        g, dx = unet.backward(theta, acts, dout, in_ch, out_ch, widths, store_bf16=store)
        n_conv = 4 * len(widths) - 2
        assert len(seen["fwd"]) == n_conv and len(seen["bwd"]) == n_conv
        checks = []
        for a, W in seen["fwd"]:
            checks += [_bf16_exact(a), _bf16_exact(W)]
        for hin, y in acts[:-1]:
            checks.append(_bf16_exact(y))                      # stored convolution outputs
        checks.append(_bf16_exact(acts[-1][0]))                 # head input
        for a, W, dy in seen["bwd"]:
            checks += [_bf16_exact(a), _bf16_exact(W), _bf16_exact(dy)]
        checks.append(_bf16_exact(dx))                          # gradient of the input
        if store:
            assert all(checks), checks
            # the head's FP32 output is not rounded
            assert not _bf16_exact(out)
        else:
            # the network input x is a BF16 value by construction; all else is not
            assert sum(checks) <= 2, checks
