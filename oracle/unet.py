"""FP64 reference of the warm-start U-Net: forward, backward, loss and Adam.

TEST INFRASTRUCTURE ONLY (see the package header).

The network is not part of the paper; its shape is fixed by this project's
specification: a 3-D U-Net with L levels of widths C_0..C_{L-1}; per level two
3x3x3 convolutions (zero padding 1) each followed by ReLU; 2x2x2 average pooling
between encoder levels; in the decoder, nearest-neighbour x2 upsampling, channel
concatenation [upsampled, skip] and two 3x3x3 convolutions + ReLU; a 1x1x1 head
without activation.  Arrays are NDHWC ``[n][z][y][x][c]``.

Convolution weights are stored as ``W[tap][c_in][c_out]`` with
``tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)``, followed by the bias ``b[c_out]``;
the flat parameter vector lists the layers in forward order (encoder levels, then
decoder levels from the deepest, then the head).

Pinned by ``tests/test_oracle_unet.py``: convolution against a per-voxel Python loop
on tiny inputs and against a centred delta kernel (identity); pooling and
upsampling identities; the parameter count of the 16-32-64-64 network (911,715);
every gradient against central finite differences in FP64; the first Adam step
moving each parameter by lr * sign(gradient).
"""

from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(x):
    """Round to the nearest BFloat16 value (ties to even), returned as float64.

    BFloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of an
    IEEE binary32 number.  The value is first rounded to binary32; rounding to nearest
    with ties to even then adds 0x7fff plus the lowest kept bit to the bit pattern and
    truncates the low 16 bits (a carry moves into the exponent, so the largest values
    round to infinity).  NaN stays NaN.  Pinned against PyTorch's CPU cast to
    ``torch.bfloat16`` in ``tests/test_oracle_unet.py``.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    with np.errstate(invalid="ignore"):          # signalling NaN patterns widen quietly
        out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def _keep(x, store):
    return bf16(x) if store else x


def layer_shapes(in_ch, out_ch, widths):
    """(c_in, c_out, taps) of every convolution, in forward order."""
    L = len(widths)
    shapes = []
    cin = in_ch
    for lvl in range(L):
        shapes.append((cin, widths[lvl], 27))
        shapes.append((widths[lvl], widths[lvl], 27))
        cin = widths[lvl]
    for lvl in range(L - 2, -1, -1):
        shapes.append((widths[lvl + 1] + widths[lvl], widths[lvl], 27))
        shapes.append((widths[lvl], widths[lvl], 27))
    shapes.append((widths[0], out_ch, 1))
    return shapes


def param_count(in_ch, out_ch, widths):
    return sum(t * ci * co + co for ci, co, t in layer_shapes(in_ch, out_ch, widths))


def unpack(theta, in_ch, out_ch, widths):
    """Split the flat parameter vector into [(W, b), ...] views."""
    out, o = [], 0
    for ci, co, t in layer_shapes(in_ch, out_ch, widths):
        W = theta[o:o + t * ci * co].reshape(t, ci, co)
        o += t * ci * co
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == len(theta)
    return out


def conv3(x, W, b):
    """3x3x3 convolution with zero padding 1: out = b + sum_tap shift(x) @ W[tap]."""
    n, D, H, Wd, ci = x.shape
    xp = np.zeros((n, D + 2, H + 2, Wd + 2, ci))
    xp[:, 1:-1, 1:-1, 1:-1, :] = x
    out = np.broadcast_to(b, (n, D, H, Wd, W.shape[2])).copy()
    for t, (dz, dy, dx) in enumerate(TAPS):
        sh = xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd, :]
        out += sh @ W[t]
    return out


def conv3_backward(x, W, dy):
    """Gradients of conv3 with respect to x, W and b."""
    n, D, H, Wd, ci = x.shape
    xp = np.zeros((n, D + 2, H + 2, Wd + 2, ci))
    xp[:, 1:-1, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for t, (dz, dyy, dx) in enumerate(TAPS):
        sl = (slice(None), slice(1 + dz, 1 + dz + D), slice(1 + dyy, 1 + dyy + H),
              slice(1 + dx, 1 + dx + Wd), slice(None))
        dW[t] = np.tensordot(xp[sl], dy, axes=([0, 1, 2, 3], [0, 1, 2, 3]))
        dxp[sl] += dy @ W[t].T
    db = dy.sum(axis=(0, 1, 2, 3))
    return dxp[:, 1:-1, 1:-1, 1:-1, :], dW, db


def conv1(x, W, b):
    return x @ W[0] + b


def pool2(x):
    n, D, H, Wd, c = x.shape
    return x.reshape(n, D // 2, 2, H // 2, 2, Wd // 2, 2, c).mean(axis=(2, 4, 6))


def pool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_backward(dy):
    n, D, H, Wd, c = dy.shape
    return dy.reshape(n, D // 2, 2, H // 2, 2, Wd // 2, 2, c).sum(axis=(2, 4, 6))


def forward(theta, x, in_ch, out_ch, widths, keep=False, store_bf16=False):
    """Network output; with keep=True also the activations needed by backward().

    store_bf16=True rounds the 3x3x3 weights and every stored activation (convolution
    outputs, pooled and upsampled tensors) to BFloat16, the storage format of the
    GPU kernels, while all arithmetic stays FP64.
    """
    layers = unpack(theta, in_ch, out_ch, widths)
    if store_bf16:
        layers = [(bf16(W), b) if W.shape[0] == 27 else (W, b) for W, b in layers]
    st = store_bf16
    L = len(widths)
    acts = []                      # (input, output) of each conv, in order
    li = 0
    h = x
    skips = []
    for lvl in range(L):
        if lvl > 0:
            h = _keep(pool2(h), st)
        for _ in range(2):
            W, b = layers[li]
            y = _keep(np.maximum(conv3(h, W, b), 0.0), st)
            acts.append((h, y))
            h = y
            li += 1
        skips.append(h)
    for lvl in range(L - 2, -1, -1):
        h = np.concatenate([up2(h), skips[lvl]], axis=-1)
        for _ in range(2):
            W, b = layers[li]
            y = _keep(np.maximum(conv3(h, W, b), 0.0), st)
            acts.append((h, y))
            h = y
            li += 1
    W, b = layers[li]
    out = conv1(h, W, b)
    acts.append((h, out))
    return (out, acts) if keep else out


def backward(theta, acts, dout, in_ch, out_ch, widths, store_bf16=False):
    """Gradient of the loss with respect to theta (and the input), given dL/dout.

    store_bf16=True uses BFloat16-rounded 3x3x3 weights and rounds every stored
    activation gradient (head input gradient, convolution input gradients,
    upsampling and pooling gradients) to BFloat16, as the GPU kernels store them.
    """
    layers = unpack(theta, in_ch, out_ch, widths)
    if store_bf16:
        layers = [(bf16(W), b) if W.shape[0] == 27 else (W, b) for W, b in layers]
    st = store_bf16
    grads = [None] * len(layers)
    L = len(widths)
    li = len(layers) - 1
    hin, _ = acts[li]
    W, _ = layers[li]
    grads[li] = (np.tensordot(hin, dout, axes=([0, 1, 2, 3], [0, 1, 2, 3]))[None],
                 dout.sum(axis=(0, 1, 2, 3)))
    dh = _keep(dout @ W[0].T, st)
    li -= 1
    dskips = [None] * L
    for lvl in range(0, L - 1):
        for _ in range(2):
            hin, y = acts[li]
            W, _ = layers[li]
            dpre = dh * (y > 0)
            dh, dW, db = conv3_backward(hin, W, dpre)
            dh = _keep(dh, st)
            grads[li] = (dW, db)
            li -= 1
        cu = widths[lvl + 1]
        dskips[lvl] = dh[..., cu:]
        dh = _keep(up2_backward(dh[..., :cu]), st)
    for lvl in range(L - 1, -1, -1):
        if lvl < L - 1:
            dh = _keep(dh + dskips[lvl], st)
        for _ in range(2):
            hin, y = acts[li]
            W, _ = layers[li]
            dpre = dh * (y > 0)
            dh, dW, db = conv3_backward(hin, W, dpre)
            dh = _keep(dh, st)
            grads[li] = (dW, db)
            li -= 1
        if lvl > 0:
            dh = pool2_backward(dh)
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()]) for g in grads])
    return flat, dh


def mse(out, target):
    """Mean squared error and its gradient with respect to out."""
    d = out - target
    return float((d * d).mean()), 2.0 * d / d.size


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), in place; t counts from 1."""
    m[:] = b1 * m + (1.0 - b1) * g
    v[:] = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    theta -= lr * mh / (np.sqrt(vh) + eps)
    return theta
