"""Exact parity of the network's data-movement kernels (pooling, upsampling and their
gradients, the 1x1x1 head and its gradient, the MSE and the input padding) against the
FP64 oracle, on small-integer data for which every FP32 sum and every BF16 value is
exact: the GPU must equal the oracle bit for bit.  Shapes are ragged (no dimension a
multiple of the kernels' natural widths) and cover several channel groups."""

import numpy as np
import pytest

from gpu_helpers import require_gpu
from oracle import unet

pytestmark = pytest.mark.gpu


def _bits(a):
    """BF16 bit patterns (int16) of values exactly representable in BF16."""
    a = np.asarray(a, dtype=np.float64)
    assert np.array_equal(unet.bf16(a), a), "test data must be exact BF16 values"
    return (a.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def _vals(t):
    """FP64 values of a GPU tensor of BF16 bit patterns."""
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _net(torch, seed=1, out_ch=3):
    from paper_2505_03067_amd import Net
    return Net(13, out_ch, [16, 32], seed=seed)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("shape,c", [((2, 6, 10, 14), 16), ((1, 2, 4, 34), 48), ((3, 4, 2, 6), 64)])
def test_pool_exact(shape, c):
    torch = require_gpu()
    import paper_2505_03067_amd.mpm as b
    rng = np.random.default_rng(c)
    x = rng.integers(-8, 9, size=shape + (c,)).astype(np.float64)
    want = unet.pool2(x)
    n, d, h, w = shape
    out = torch.empty((n, d // 2, h // 2, w // 2, c), dtype=torch.int16, device="cuda")
    net = _net(torch)
    net.debug_op(b.MPM_OP_POOL, shape, c, 0, _dev(torch, _bits(x)), None, out)
    net.close()
    assert np.array_equal(_vals(out), want)


@pytest.mark.parametrize("shape,c,c2", [((2, 6, 10, 14), 16, 48), ((1, 4, 4, 18), 32, 32),
                                        ((1, 2, 2, 2), 64, 0)])
def test_pool_backward_add_exact(shape, c, c2):
    """Gradient of the pooling (an eighth of the parent's gradient to each child) plus
    the skip gradient, which is the last c of the c2 channels of a decoder
    concatenation's gradient; c2 = 0: no skip."""
    torch = require_gpu()
    import paper_2505_03067_amd.mpm as b
    rng = np.random.default_rng(c + c2)
    n, d, h, w = shape
    dp = rng.integers(-16, 17, size=(n, d // 2, h // 2, w // 2, c)).astype(np.float64)
    want = unet.pool2_backward(dp)
    skip_t = None
    if c2:
        skip = rng.integers(-8, 9, size=shape + (c2,)).astype(np.float64)
        want = want + skip[..., c2 - c:]
        skip_t = _dev(torch, _bits(skip))
    out = torch.empty(shape + (c,), dtype=torch.int16, device="cuda")
    net = _net(torch)
    net.debug_op(b.MPM_OP_POOL_BWD_ADD, shape, c, c2, _dev(torch, _bits(dp)), skip_t, out)
    net.close()
    assert np.array_equal(_vals(out), want)


@pytest.mark.parametrize("shape,c,c2", [((2, 6, 10, 14), 32, 16), ((1, 4, 2, 30), 64, 64), ((1, 2, 2, 2), 16, 16)])
def test_upsample_concat_and_its_gradient_exact(shape, c, c2):
    torch = require_gpu()
    import paper_2505_03067_amd.mpm as b
    rng = np.random.default_rng(3 * c + c2)
    n, d, h, w = shape
    # any finite BF16 values: the forward is a copy of 16-byte words
    hh = unet.bf16(rng.normal(scale=10.0, size=(n, d // 2, h // 2, w // 2, c)))
    skip = unet.bf16(rng.normal(size=shape + (c2,)))
    cat = torch.empty(shape + (c + c2,), dtype=torch.int16, device="cuda")
    net = _net(torch)
    net.debug_op(b.MPM_OP_UP2_CAT, shape, c, c2, _dev(torch, _bits(hh)), _dev(torch, _bits(skip)), cat)
    want = np.concatenate([unet.up2(hh), skip], axis=-1)
    assert np.array_equal(_vals(cat), want)
    # gradient: the first c channels of the concatenation's gradient, summed over children
    dcat = rng.integers(-16, 17, size=shape + (c + c2,)).astype(np.float64)
    dh = torch.empty((n, d // 2, h // 2, w // 2, c), dtype=torch.int16, device="cuda")
    net.debug_op(b.MPM_OP_UP2_BWD, shape, c, c2, _dev(torch, _bits(dcat)), None, dh)
    net.close()
    assert np.array_equal(_vals(dh), unet.up2_backward(dcat[..., :c]))


@pytest.mark.parametrize("out_ch,shape", [(3, (2, 8, 8, 16)), (4, (1, 3, 5, 7)), (1, (1, 1, 1, 9))])
def test_head_and_its_gradient_exact(out_ch, shape):
    torch = require_gpu()
    import paper_2505_03067_amd.mpm as b
    rng = np.random.default_rng(out_ch)
    net = _net(torch, out_ch=out_ch)
    theta = np.zeros(net.count, np.float32)
    layers = unet.unpack(theta, 13, out_ch, [16, 32])
    Wh, bh = layers[-1]
    Wh[:] = rng.integers(-2, 3, size=Wh.shape)
    bh[:] = rng.integers(-3, 4, size=bh.shape)
    net.set_params(torch.from_numpy(theta).cuda())
    P = int(np.prod(shape))
    hin = rng.integers(-3, 4, size=(P, 16)).astype(np.float64)
    out = torch.empty((P, out_ch), dtype=torch.float32, device="cuda")
    net.debug_op(b.MPM_OP_HEAD, shape, 16, 0, _dev(torch, _bits(hin)), None, out)
    W64 = Wh.astype(np.float64)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), unet.conv1(hin, W64, bh.astype(np.float64)))
    dout = rng.integers(-4, 5, size=(P, out_ch)).astype(np.float32)
    dh = torch.empty((P, 16), dtype=torch.int16, device="cuda")
    gpar = torch.empty(16 * out_ch + out_ch, dtype=torch.float32, device="cuda")
    net.debug_op(b.MPM_OP_HEAD_BWD, shape, 16, 0, _dev(torch, _bits(hin)), _dev(torch, dout), dh, gpar)
    net.close()
    d64 = dout.astype(np.float64)
    assert np.array_equal(_vals(dh), d64 @ W64[0].T)
    want = np.concatenate([(hin.T @ d64).ravel(), d64.sum(axis=0)])
    assert np.array_equal(gpar.cpu().numpy().astype(np.float64), want)


@pytest.mark.parametrize("c,cp,P", [(13, 16, 1000), (17, 32, 77), (8, 16, 5)])
def test_pad_channels_exact(c, cp, P):
    torch = require_gpu()
    import paper_2505_03067_amd.mpm as b
    rng = np.random.default_rng(c)
    x = unet.bf16(rng.normal(size=(P, c)))
    out = torch.full((P, cp), 12345, dtype=torch.int16, device="cuda")
    net = _net(torch)
    net.debug_op(b.MPM_OP_PAD, (1, 1, 1, P), c, cp, _dev(torch, _bits(x)), None, out)
    net.close()
    want = np.zeros((P, cp))
    want[:, :c] = x
    assert np.array_equal(_vals(out), want)


@pytest.mark.parametrize("count", [4096, 2 ** 20, 3 * 2 ** 16])
def test_mse_exact(count):
    """grad = 2 (out - target) / count and the mean squared error; with integer data and a
    count of the form 2^k or 3 2^k the FP32 gradient is exact or rounded once (compared
    with the oracle's value rounded to FP32), the FP64 loss exact."""
    torch = require_gpu()
    rng = np.random.default_rng(count % 97)
    out = rng.integers(-50, 51, size=count).astype(np.float32)
    tgt = rng.integers(-50, 51, size=count).astype(np.float32)
    net = _net(torch)
    g = torch.empty(count, dtype=torch.float32, device="cuda")
    loss = net.mse(_dev(torch, out), _dev(torch, tgt), g)
    net.close()
    want_loss, want_g = unet.mse(out.astype(np.float64), tgt.astype(np.float64))
    assert loss == want_loss
    # the kernel multiplies by the FP32 value of 2 / count: the same as the oracle's
    # gradient when 2 / count is a power of two, else within one FP32 rounding
    got_g = g.cpu().numpy().astype(np.float64)
    if count & (count - 1) == 0:
        assert np.array_equal(got_g, want_g)
    else:
        assert np.max(np.abs(got_g - want_g) / np.maximum(np.abs(want_g), 1e-300)) <= 2.0 ** -22
