"""GPU parity of the warm-start U-Net kernels against the FP64 oracle.

Three levels: (1) single layers and every data-movement kernel on small-integer data,
where FP32 accumulation is exact, bit for bit (here and in test_gpu_unet_ops.py);
(2) every step of a whole forward and backward pass against the oracle fed the GPU's
own stored BF16 tensors, relative L2 error <= 1e-3; (3) the whole network against the
BF16-storage oracle (FP64 arithmetic, BF16 rounding of weights, activations and
activation gradients where the GPU stores them), with bars derived from the oracle's
own spread between FP64 and FP32 accumulation.
"""

import numpy as np
import pytest

from gpu_helpers import require_gpu
from oracle import unet

pytestmark = pytest.mark.gpu


def _bf16_bits(a):
    """Bit patterns of BF16 values that are exactly representable (a = unet.bf16(...))."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32)
    return (u >> 16).astype(np.uint16)


def _run(widths, shape, seed, in_ch=13, out_ch=3):
    torch = require_gpu()
    from paper_2505_03067_amd import Net
    rng = np.random.default_rng(seed)
    n, d, h, w = shape
    net = Net(in_ch, out_ch, widths, seed=seed)
    P = net.count
    assert P == unet.param_count(in_ch, out_ch, widths)
    theta = np.empty(P, np.float32)
    # He-scaled weights (activations stay of order one through the depth) and small
    # positive biases that keep most ReLUs open
    for W, b in unet.unpack(theta, in_ch, out_ch, widths):
        W[:] = rng.normal(scale=np.sqrt(2.0 / (W.shape[0] * W.shape[1])), size=W.shape)
        b[:] = np.abs(rng.normal(scale=0.05, size=b.shape))
    net.set_params(torch.from_numpy(theta).cuda())
    x = unet.bf16(rng.uniform(-1, 1, size=(n, d, h, w, in_ch)))
    xg = torch.from_numpy(_bf16_bits(x).view(np.int16)).cuda()
    out = torch.empty((n, d, h, w, out_ch), dtype=torch.float32, device="cuda")
    net.forward(xg, out)
    target = rng.normal(size=(n, d, h, w, out_ch)).astype(np.float32)
    tg = torch.from_numpy(target).cuda()
    gout = torch.empty_like(out)
    loss_gpu = net.mse(out, tg, gout)
    net.zero_grad()
    net.backward(gout)
    grads = net.grads().cpu().numpy().astype(np.float64)
    outg = out.cpu().numpy().astype(np.float64)
    net.close()
    th = theta.astype(np.float64)
    ref, acts = unet.forward(th, x, in_ch, out_ch, widths, keep=True, store_bf16=True)
    loss_ref, dref = unet.mse(ref, target.astype(np.float64))
    gref, _ = unet.backward(th, acts, dref, in_ch, out_ch, widths, store_bf16=True)
    return outg, ref, grads, gref, loss_gpu, loss_ref, th, x, target


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# Tap orders of the FP32-accumulating oracle variants: natural, reversed, even taps then
# odd taps, centre tap first.  Each is another order of the same FP32 sums.
TAP_ORDERS = [list(range(27)), list(range(26, -1, -1)), list(range(0, 27, 2)) + list(range(1, 27, 2)),
              [13] + [t for t in range(27) if t != 13]]


def _conv3_f32(order):
    """conv3 with FP32 storage and FP32 accumulation over the taps in 'order'."""
    def conv(a, W, b):
        a32, W32 = a.astype(np.float32), W.astype(np.float32)
        n, D, H, Wd, ci = a.shape
        xp = np.zeros((n, D + 2, H + 2, Wd + 2, ci), np.float32)
        xp[:, 1:-1, 1:-1, 1:-1, :] = a32
        out = np.broadcast_to(np.asarray(b, np.float32), (n, D, H, Wd, W.shape[2])).copy()
        for t in order:
            dz, dy, dx = unet.TAPS[t]
            out += xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd, :] @ W32[t]
        return out.astype(np.float64)
    return conv


def _conv3_backward_f32(order):
    """conv3_backward with FP32 storage and FP32 accumulation over the taps in 'order'."""
    def conv_b(a, W, g):
        a32, W32, g32 = a.astype(np.float32), W.astype(np.float32), g.astype(np.float32)
        n, D, H, Wd, ci = a.shape
        xp = np.zeros((n, D + 2, H + 2, Wd + 2, ci), np.float32)
        xp[:, 1:-1, 1:-1, 1:-1, :] = a32
        dxp = np.zeros_like(xp)
        dW = np.zeros(W.shape, np.float32)
        for t in order:
            dz, dyy, dx = unet.TAPS[t]
            sl = (slice(None), slice(1 + dz, 1 + dz + D), slice(1 + dyy, 1 + dyy + H),
                  slice(1 + dx, 1 + dx + Wd), slice(None))
            dW[t] = np.tensordot(xp[sl], g32, axes=([0, 1, 2, 3], [0, 1, 2, 3]))
            dxp[sl] += g32 @ W32[t].T
        db = g32.sum(axis=(0, 1, 2, 3), dtype=np.float32)
        return (dxp[:, 1:-1, 1:-1, 1:-1, :].astype(np.float64), dW.astype(np.float64), db.astype(np.float64))
    return conv_b


def _oracle_fp32_accumulation(th, x, target, widths, monkeypatch, order):
    """The BF16-storage oracle with its convolutions accumulated in FP32 (taps in
    'order') instead of FP64: output and parameter gradient of an implementation that
    stores what the GPU stores and accumulates in FP32, in another order than the GPU's.
    Its distance to the FP64-accumulating oracle is the spread that BF16 rounding flips
    and ReLU gate flips alone produce, whatever the kernels do."""
    with monkeypatch.context() as mp:
        mp.setattr(unet, "conv3", _conv3_f32(order))
        mp.setattr(unet, "conv3_backward", _conv3_backward_f32(order))
        out, acts = unet.forward(th, x, 13, 3, widths, keep=True, store_bf16=True)
        _, dout = unet.mse(out, target.astype(np.float64))
        g, _ = unet.backward(th, acts, dout, 13, 3, widths, store_bf16=True)
    return out, g


def _per_layer(widths, a, b):
    errs, o = [], 0
    for ci, co, t in unet.layer_shapes(13, 3, widths):
        nw = t * ci * co
        errs.append(max(_rel(a[o:o + nw], b[o:o + nw]), _rel(a[o + nw:o + nw + co], b[o + nw:o + nw + co])))
        o += nw + co
    return errs


# the first decoder convolution of each level reads the upsampled deeper output and the
# skip directly (for [16, 48] the upsampled input is three 16-channel chunks)
@pytest.mark.parametrize("widths,shape", [([16, 32], (2, 8, 8, 16)), ([16, 32, 64, 64], (1, 16, 16, 16)),
                                          ([16, 32, 64, 64], (2, 8, 16, 24)), ([16, 48], (1, 6, 8, 18)),
                                          ([16, 16, 32, 32], (1, 16, 16, 16))])
def test_forward_backward_match_oracle(widths, shape, monkeypatch):
    """The whole network against the BF16-storage oracle.  Both round to BF16 at the
    same points, so they differ only where an FP32 sum and an FP64 sum round to
    different BF16 values (one unit in the last place) or fall on different sides of a
    ReLU.  Such a flip changes the 27 C_out outputs that read the voxel slightly, some of
    those cross a rounding boundary in turn, and the differences spread layer after
    layer, furthest into the gradients of the first layers: for [16, 32] on 2 x 8 x 8 x 16
    the GPU's first layer differs from the oracle in 2 of 32,768 stored values and the
    sixth in 6.5%.  How far that goes depends on where the first flips fall, so an
    end-to-end comparison is not a parity bar for the kernels; the survey's 1e-3 is
    applied per step, on the GPU's own inputs, by test_layerwise_chain_matches_oracle
    (and exactly, on integer data, by test_single_layer_kernels_exact and
    test_gpu_unet_ops.py).  Here the output, the loss and the whole gradient must agree
    to within max(bar, 4 x the largest spread of four FP32-accumulating variants of the
    oracle with the taps in different orders), with bars 5e-3 for the output and the
    loss and 2e-2 for the gradient, and the
    gradient's direction to a cosine of 0.999; per-layer gradient errors are printed."""
    outg, ref, grads, gref, loss_gpu, loss_ref, th, x, target = _run(widths, shape, seed=len(widths) * 7 + shape[1])
    s_out, s_loss, s_layers, s_all = 0.0, 0.0, None, 0.0
    for order in TAP_ORDERS:
        alt_out, alt_g = _oracle_fp32_accumulation(th, x, target, widths, monkeypatch, order)
        loss_alt, _ = unet.mse(alt_out, target.astype(np.float64))
        s_out = max(s_out, _rel(alt_out, ref))
        s_loss = max(s_loss, abs(loss_alt - loss_ref) / loss_ref)
        sl = _per_layer(widths, alt_g, gref)
        s_layers = sl if s_layers is None else [max(a, c) for a, c in zip(s_layers, sl)]
        s_all = max(s_all, _rel(alt_g, gref))
    e_out = _rel(outg, ref)
    print(f"output rel err {e_out:.2e}, oracle FP32-accumulation spread {s_out:.2e}")
    errs = _per_layer(widths, grads, gref)
    for li, (ci, co, t) in enumerate(unet.layer_shapes(13, 3, widths)):
        print(f"layer {li} ({ci}->{co}, {t} taps): gradient rel err {errs[li]:.2e}, "
              f"oracle FP32-accumulation spread {s_layers[li]:.2e}")
    e_all = _rel(grads, gref)
    cos = float(grads @ gref / (np.linalg.norm(grads) * np.linalg.norm(gref)))
    print(f"whole gradient rel err {e_all:.2e}, spread {s_all:.2e}, cosine {cos:.6f}")
    assert e_out <= max(5e-3, 4 * s_out)
    assert abs(loss_gpu - loss_ref) <= max(5e-3, 4 * s_loss) * loss_ref
    assert e_all <= max(2e-2, 4 * s_all)
    assert cos >= 0.999
    # against the plain FP64 network the difference is at BF16 level
    plain = unet.forward(th, x, 13, 3, widths)
    assert _rel(outg, plain) <= 3e-2


@pytest.mark.parametrize("widths,shape", [([16, 32], (2, 8, 8, 16)), ([16, 32, 64, 64], (1, 64, 64, 128)),
                                          ([16, 16, 32, 32], (1, 32, 48, 64))])
def test_inference_pass_matches_forward(widths, shape):
    """mpm_net_infer (the head fused into the last convolution's epilogue, whose output is
    then not stored) gives the forward pass's output bit for bit, on a grid small enough
    for the register-staged kernel and on one large enough for the asynchronously staged
    one; no backward pass may follow it until the next plain forward pass."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    import paper_2505_03067_amd.mpm as b
    net = m.Net(16, 3, widths, seed=21)
    g = torch.Generator().manual_seed(5)
    x = torch.randn(tuple(shape) + (16,), generator=g).to(torch.bfloat16).view(torch.int16).cuda()
    out_f = torch.empty(tuple(shape) + (3,), dtype=torch.float32, device="cuda")
    out_i = torch.full_like(out_f, float("nan"))
    net.forward(x, out_f)
    net.forward(x, out_i, infer=True)
    assert float(out_f.abs().sum()) > 0.0
    assert torch.equal(out_f.view(torch.int32), out_i.view(torch.int32))
    with pytest.raises(b.MpmError):
        net.backward(torch.zeros_like(out_f))
    with pytest.raises(b.MpmError):
        net.debug_tensor(b.MPM_NT_ACT, 4 * len(widths) - 3)   # the last 3x3x3 layer's output
    net.forward(x, out_f)
    net.zero_grad()
    net.backward(torch.zeros_like(out_f))
    net.close()


@pytest.mark.parametrize("widths,shape", [([16, 32, 64, 64], (2, 8, 16, 24)), ([16, 32, 64, 64], (1, 128, 128, 128)),
                                          ([16, 32, 48], (1, 8, 12, 20)), ([16, 16, 32, 32], (1, 32, 48, 64))])
def test_fused_pooling_matches_pool_kernel(widths, shape):
    """The pooling each encoder level's second convolution does in its epilogue equals
    k_pool2 (MPM_OP_POOL) on the stored BF16 output bit for bit: grids that leave
    partial voxel tiles, the 128^3 grid (the asynchronously staged kernel at the first
    level, the chunk-staged kernel with two output tiles at the second), and a
    three-level net."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    import paper_2505_03067_amd.mpm as b
    net = m.Net(16, 3, widths, seed=23)
    g = torch.Generator().manual_seed(9)
    x = torch.randn(tuple(shape) + (16,), generator=g).to(torch.bfloat16).view(torch.int16).cuda()
    out = torch.empty(tuple(shape) + (3,), dtype=torch.float32, device="cuda")
    net.forward(x, out)
    n, d, h, w = shape
    for lvl in range(1, len(widths)):
        fine = (n, d >> (lvl - 1), h >> (lvl - 1), w >> (lvl - 1))
        c = widths[lvl - 1]
        act = net.debug_tensor(b.MPM_NT_ACT, 2 * (lvl - 1) + 1)
        got = net.debug_tensor(b.MPM_NT_POOLED, lvl)
        want = torch.empty_like(got)
        net.debug_op(b.MPM_OP_POOL, fine, c, 0, act, None, want)
        assert got.abs().sum() > 0
        assert torch.equal(got, want), lvl
    net.close()


def _tensor(net, kind, index, shape, ch):
    t = net.debug_tensor(kind, index).cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return t.view(np.float32).astype(np.float64).reshape(tuple(shape) + (ch,))


@pytest.mark.parametrize("widths,shape", [([16, 32], (2, 8, 8, 16)), ([16, 32, 64, 64], (1, 16, 16, 16)),
                                          ([16, 32, 64, 64], (2, 8, 16, 24))])
def test_layerwise_chain_matches_oracle(widths, shape):
    """Every step of the GPU's forward and backward pass against the oracle fed the
    GPU's own stored BF16 tensors: each convolution's output, weight and bias gradients
    and stored input gradient, each pooling, concatenation, upsampling gradient and
    pooling-gradient-plus-skip, the head and the loss gradient.  From identical inputs
    the two differ only by FP32 against FP64 accumulation (and the rare BF16 rounding it
    flips), so each is held to a relative L2 error of 1e-3."""
    torch = require_gpu()
    import paper_2505_03067_amd.mpm as b
    from paper_2505_03067_amd import Net
    seed = 5 + len(widths)
    rng = np.random.default_rng(seed)
    n, d, h, w = shape
    L = len(widths)
    in_ch, out_ch = 13, 3
    net = Net(in_ch, out_ch, widths, seed=seed)
    theta = np.empty(net.count, np.float32)
    for W, bias in unet.unpack(theta, in_ch, out_ch, widths):
        W[:] = rng.normal(scale=np.sqrt(2.0 / (W.shape[0] * W.shape[1])), size=W.shape)
        bias[:] = rng.normal(scale=0.05, size=bias.shape)
    net.set_params(torch.from_numpy(theta).cuda())
    x = unet.bf16(rng.uniform(-1, 1, size=(n, d, h, w, in_ch)))
    out = torch.empty((n, d, h, w, out_ch), dtype=torch.float32, device="cuda")
    net.forward(torch.from_numpy(_bf16_bits(x).view(np.int16)).cuda(), out)
    target = rng.normal(size=(n, d, h, w, out_ch)).astype(np.float32)
    gout = torch.empty_like(out)
    net.mse(out, torch.from_numpy(target).cuda(), gout)
    net.zero_grad()
    net.backward(gout)
    grads = net.grads().cpu().numpy().astype(np.float64)
    outg = out.cpu().numpy().astype(np.float64)
    goutg = gout.cpu().numpy().astype(np.float64)

    shapes = unet.layer_shapes(in_ch, out_ch, widths)
    nl = len(shapes)
    lvl_of = [l for l in range(L) for _ in range(2)] + [l for l in range(L - 2, -1, -1) for _ in range(2)]
    grid = lambda lvl: (n, d >> lvl, h >> lvl, w >> lvl)
    acts = [_tensor(net, b.MPM_NT_ACT, li, grid(lvl_of[li]), shapes[li][1]) for li in range(nl - 1)]
    gacts = [_tensor(net, b.MPM_NT_ACT_GRAD, li, grid(lvl_of[li]), shapes[li][1]) for li in range(nl - 2)]
    gacts.append(_tensor(net, b.MPM_NT_HEAD_GRAD, 0, grid(0), widths[0]))
    xin = _tensor(net, b.MPM_NT_INPUT, 0, grid(0), 16)
    pooled = {l: _tensor(net, b.MPM_NT_POOLED, l, grid(l), widths[l - 1]) for l in range(1, L)}
    cat = {l: _tensor(net, b.MPM_NT_CAT, l, grid(l), widths[l + 1] + widths[l]) for l in range(L - 1)}
    dcat = {l: _tensor(net, b.MPM_NT_CAT_GRAD, l, grid(l), widths[l + 1] + widths[l]) for l in range(L - 1)}
    net.close()

    layers = unet.unpack(theta.astype(np.float64), in_ch, out_ch, widths)
    bar = 1e-3
    report = []

    def check(name, got, want, tol=bar):
        e = _rel(got, want)
        diff = float(np.mean(np.asarray(got) != np.asarray(want)))
        report.append(f"{name}: rel err {e:.2e}, elements that differ {diff:.2e}")
        assert e <= tol, (name, e)

    # input padding is a copy
    assert np.array_equal(xin[..., :in_ch], x) and not xin[..., in_ch:].any()
    # head and loss gradient (FP32 on the GPU)
    Wh, bh = layers[-1]
    check("head output", outg, unet.conv1(acts[-1], Wh, bh), 1e-6)
    _, g_ref = unet.mse(outg, target.astype(np.float64))
    check("loss gradient", goutg, g_ref, 1e-6)
    check("head input gradient", gacts[-1], unet.bf16(goutg @ Wh[0].T))
    o_head = sum(t * ci * co + co for ci, co, t in shapes[:-1])
    dWh = np.tensordot(acts[-1], goutg, axes=([0, 1, 2, 3], [0, 1, 2, 3]))
    check("head parameter gradient", grads[o_head:], np.concatenate([dWh.ravel(), goutg.sum(axis=(0, 1, 2, 3))]), 1e-5)

    o = 0
    for li in range(nl - 1):
        ci, co, _ = shapes[li]
        W, bias = layers[li]
        Wb = unet.bf16(W)
        lvl = lvl_of[li]
        enc = li < 2 * L
        first = li % 2 == 0
        if enc and first:
            xl = xin[..., :in_ch] if lvl == 0 else pooled[lvl]
            if lvl > 0:
                check(f"pooling into level {lvl}", pooled[lvl], unet.bf16(unet.pool2(acts[li - 1])))
        elif not enc and first:
            xl = cat[lvl]
            assert np.array_equal(cat[lvl], np.concatenate([unet.up2(acts[li - 1]), acts[2 * lvl + 1]], axis=-1))
        else:
            xl = acts[li - 1]
        check(f"layer {li} forward", acts[li], unet.bf16(np.maximum(unet.conv3(xl, Wb, bias), 0.0)))
        dpre = gacts[li] * (acts[li] > 0)
        dx, dW, db = unet.conv3_backward(xl, Wb, dpre)
        nw = 27 * ci * co
        check(f"layer {li} weight gradient", grads[o:o + nw], dW.ravel())
        check(f"layer {li} bias gradient", grads[o + nw:o + nw + co], db)
        o += nw + co
        if enc and not first:
            check(f"layer {li} input gradient", gacts[li - 1], unet.bf16(dx))
        elif not enc and not first:
            check(f"layer {li} input gradient", gacts[li - 1], unet.bf16(dx))
        elif not enc and first:
            check(f"layer {li} input gradient (concatenation)", dcat[lvl], unet.bf16(dx))
            cu = widths[lvl + 1]
            check(f"upsampling gradient into layer {li - 1}", gacts[li - 1],
                  unet.bf16(unet.up2_backward(dcat[lvl][..., :cu])))
        elif lvl > 0:
            # gradient of the pooled input, then the pooling gradient plus the skip's
            want = unet.bf16(unet.pool2_backward(unet.bf16(dx)) + dcat[lvl - 1][..., widths[lvl]:])
            check(f"pooling gradient + skip into layer {li - 1}", gacts[li - 1], want)
    print("\n".join(report))


@pytest.mark.parametrize("widths,li,shape", [([16, 32], 0, (2, 8, 8, 16)), ([16, 32], 1, (1, 8, 6, 16)),
                                             ([16, 32], 2, (1, 4, 4, 8)), ([16, 32], 4, (2, 8, 8, 8)),
                                             ([16, 32], 3, (1, 5, 9, 35)),
                                             ([16, 32, 64, 64], 4, (1, 6, 7, 20)),
                                             ([16, 32, 64, 64], 8, (1, 8, 8, 16)),
                                             ([16, 32, 64, 64], 10, (2, 4, 5, 17)),
                                             ([16, 32], 1, (1, 64, 64, 64)), ([16, 32], 3, (1, 32, 64, 64)),
                                             ([16, 32], 3, (1, 64, 64, 64)), ([16, 32], 1, (2, 64, 64, 64))])
def test_single_layer_kernels_exact(widths, li, shape):
    """Forward, input-gradient and weight-gradient kernels of one layer on small-integer
    data, for which FP32 accumulation is exact: the GPU must equal the FP64 oracle
    bit for bit (catches any index, tap or layout error).  The largest grids give the
    persistent convolution blocks several work items each, and the weight-gradient
    blocks several voxel tiles each; the 32-channel layer on 64^3 runs the variant with
    two output tiles per block, and the 16-channel layer on two 64^3 samples the one
    that stages its input tiles asynchronously."""
    torch = require_gpu()
    from paper_2505_03067_amd import Net
    net = Net(13, 3, widths, seed=3)
    rng = np.random.default_rng(li)
    P = net.count
    theta = np.zeros(P, np.float32)
    for W, b in unet.unpack(theta, 13, 3, widths):
        W[:] = rng.integers(-2, 3, size=W.shape)
        b[:] = rng.integers(-3, 4, size=b.shape)
    net.set_params(torch.from_numpy(theta).cuda())
    ci, co, _ = unet.layer_shapes(13, 3, widths)[li]
    W, b = unet.unpack(theta.astype(np.float64), 13, 3, widths)[li]
    cip = (ci + 15) // 16 * 16
    n, d, h, w = shape
    x = np.zeros((n, d, h, w, cip))
    x[..., :ci] = rng.integers(-2, 3, size=(n, d, h, w, ci))
    g = rng.integers(-3, 4, size=(n, d, h, w, co)).astype(np.float64)
    gate = rng.integers(-1, 2, size=(n, d, h, w, co)).astype(np.float64)   # -1, 0, 1
    xb = torch.from_numpy(_bf16_bits(x).view(np.int16)).cuda()
    gb = torch.from_numpy(_bf16_bits(g).view(np.int16)).cuda()
    gtb = torch.from_numpy(_bf16_bits(gate).view(np.int16)).cuda()
    out0 = torch.empty((n, d, h, w, co), dtype=torch.float32, device="cuda")
    out1 = torch.empty((n, d, h, w, ci), dtype=torch.float32, device="cuda")
    out2 = torch.empty((27, ci, co), dtype=torch.float32, device="cuda")
    net.debug_layer(li, 0, xb, None, None, out0)
    net.debug_layer(li, 1, None, gb, gtb, out1)
    net.debug_layer(li, 2, xb, gb, gtb, out2)
    net.close()
    want0 = unet.conv3(x[..., :ci], W, b)
    gg = g * (gate > 0)
    want1, want2, _ = unet.conv3_backward(x[..., :ci], W, gg)
    assert np.array_equal(out0.cpu().numpy().astype(np.float64), want0)
    assert np.array_equal(out1.cpu().numpy().astype(np.float64), want1)
    assert np.array_equal(out2.cpu().numpy().astype(np.float64), want2)


def test_full_grid_forward_sampled():
    """The 16-32-64-64 network's forward pass on a 128^3 grid (the warm start's box grid),
    where the launches take their production shapes: the 128^3 layers with 16 inputs
    and outputs stage their input tiles asynchronously, the 64^3 layers with 32 outputs
    run two output tiles per block, and the decoder's first layer there reads the
    upsampled deeper output and the skip directly.  Those layers are recomputed by the oracle at
    sampled voxels (the grid's corners and some face voxels among them) from the GPU's
    own stored BF16 inputs and held to the layerwise bar: relative L2 error 1e-3."""
    torch = require_gpu()
    import paper_2505_03067_amd.mpm as b
    from paper_2505_03067_amd import Net
    widths, in_ch, out_ch, S = [16, 32, 64, 64], 16, 3, 128
    rng = np.random.default_rng(21)
    net = Net(in_ch, out_ch, widths, seed=21)
    theta = np.empty(net.count, np.float32)
    for W, bias in unet.unpack(theta, in_ch, out_ch, widths):
        W[:] = rng.normal(scale=np.sqrt(2.0 / (W.shape[0] * W.shape[1])), size=W.shape)
        bias[:] = rng.normal(scale=0.05, size=bias.shape)
    net.set_params(torch.from_numpy(theta).cuda())
    x = unet.bf16(rng.uniform(-1, 1, size=(1, S, S, S, in_ch)))
    out = torch.empty((1, S, S, S, out_ch), dtype=torch.float32, device="cuda")
    net.forward(torch.from_numpy(_bf16_bits(x).view(np.int16)).cuda(), out)
    shapes = unet.layer_shapes(in_ch, out_ch, widths)
    lvl_of = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0]
    keep = [0, 1, 2, 3, 9, 10, 11, 12, 13]
    acts = {li: _tensor(net, b.MPM_NT_ACT, li, (1,) + (S >> lvl_of[li],) * 3, shapes[li][1]) for li in keep}
    net.close()
    layers = unet.unpack(theta.astype(np.float64), in_ch, out_ch, widths)

    def sampled(xl, li, k):
        n = xl.shape[1]
        pts = rng.integers(0, n, size=(k, 3))
        pts = np.concatenate([pts, [[z, y, xx] for z in (0, n - 1) for y in (0, n - 1) for xx in (0, n - 1)],
                              [[0, n // 2, 3], [n - 1, 5, n // 2], [7, 0, n - 1]]])
        xp = np.zeros((n + 2, n + 2, n + 2, xl.shape[-1]))
        xp[1:-1, 1:-1, 1:-1] = xl[0]
        patches = np.stack([xp[z:z + 3, y:y + 3, xx:xx + 3] for z, y, xx in pts])
        W, bias = layers[li]
        want = unet.bf16(np.maximum(unet.conv3(patches, unet.bf16(W), bias)[:, 1, 1, 1], 0.0))
        got = acts[li][0][pts[:, 0], pts[:, 1], pts[:, 2]]
        return got, want

    for li, xl in ((1, acts[0]), (3, acts[2]), (11, acts[10]), (13, acts[12])):
        got, want = sampled(xl, li, 400)
        assert _rel(got, want) <= 1e-3, (li, _rel(got, want))
    # decoder level 1, first layer: upsampled level-2 output concatenated with the skip
    cat = np.concatenate([unet.up2(acts[9]), acts[3]], axis=-1)
    got, want = sampled(cat, 10, 400)
    assert _rel(got, want) <= 1e-3, (10, _rel(got, want))


def test_adam_step_matches_oracle():
    torch = require_gpu()
    from paper_2505_03067_amd import Net
    net = Net(13, 3, [16, 32], seed=5)
    rng = np.random.default_rng(9)
    th = rng.normal(scale=0.1, size=net.count).astype(np.float32)
    g = rng.normal(size=net.count).astype(np.float32)
    net.set_params(torch.from_numpy(th).cuda())
    net.set_grads(torch.from_numpy(g).cuda())
    m = np.zeros(net.count)
    v = np.zeros(net.count)
    want = th.astype(np.float64).copy()
    for t in (1, 2, 3):
        net.adam(1e-3, t)
        unet.adam(want, g.astype(np.float64), m, v, t, lr=1e-3)
    got = net.params().cpu().numpy().astype(np.float64)
    net.close()
    assert np.max(np.abs(got - want)) <= 1e-6
