"""FP64 numpy reference of the surrogate network's layers.

TEST INFRASTRUCTURE ONLY: the GPU parity tests and the training-gradient
checks compare the gfx950 kernels with these definitions; the product path
never imports this module.

Conventions (channels-last): activations x[n, d, h, w, c]; convolution weights
W[co, taps * ci] with tap = (dz+1)*9 + (dy+1)*3 + (dx+1) for a 3x3x3 kernel
(one tap, offset 0, for 1x1x1); stride 1, "same" output size; outside the box
the input is zero, or wraps on the axes named in the periodic mask (bit 0 x,
1 y, 2 z).  The convolution is the cross-correlation
    y[p, o] = b[o] + sum_t sum_c W[o, t*ci + c] x[p + off(t), c].
"""
from __future__ import annotations

import numpy as np


def tap_offsets(k):
    if k == 1:
        return [(0, 0, 0)]
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x, dz, dy, dx, pmask):
    """s[p] = x[p + (dz, dy, dx)], zero or periodic beyond the box."""
    out = x
    for axis, off, bit in ((1, dz, 4), (2, dy, 2), (3, dx, 1)):
        if off == 0:
            continue
        if pmask & bit:
            out = np.roll(out, -off, axis=axis)
        else:
            rolled = np.roll(out, -off, axis=axis)
            idx = [slice(None)] * out.ndim
            idx[axis] = slice(out.shape[axis] - off, None) if off > 0 else slice(0, -off)
            rolled[tuple(idx)] = 0.0
            out = rolled
    return out


def conv3d(x, W, bias=None, k=3, pmask=0):
    n, d, h, w, ci = x.shape
    co = W.shape[0]
    offs = tap_offsets(k)
    Wr = W.reshape(co, len(offs), ci)
    y = np.zeros((n, d, h, w, co))
    for t, (dz, dy, dx) in enumerate(offs):
        y += np.einsum("ndhwc,oc->ndhwo", shift(x, dz, dy, dx, pmask), Wr[:, t, :])
    if bias is not None:
        y += bias
    return y


def conv3d_at(x, W, points, bias=None, k=3, pmask=0):
    """The convolution's definition evaluated at selected output positions
    only (points: (m, 4) integer array of (n, z, y, x)), for layers too large
    to evaluate whole: y[p, o] = b[o] + sum_t sum_c W[o, t*ci + c] x[p + off(t), c]."""
    n, d, h, w, ci = x.shape
    co = W.shape[0]
    offs = tap_offsets(k)
    Wr = W.reshape(co, len(offs), ci)
    out = np.zeros((len(points), co))
    for j, (b, z, y, xx) in enumerate(np.asarray(points)):
        acc = np.zeros(co) if bias is None else np.array(bias, dtype=np.float64)
        for t, (dz, dy, dx) in enumerate(offs):
            q = [z + dz, y + dy, xx + dx]
            ok = True
            for a, (size, bit) in enumerate(((d, 4), (h, 2), (w, 1))):
                if q[a] < 0 or q[a] >= size:
                    if pmask & bit:
                        q[a] %= size
                    else:
                        ok = False
            if ok:
                acc = acc + Wr[:, t, :] @ x[b, q[0], q[1], q[2], :]
        out[j] = acc
    return out


def conv3d_bwd_data(dy, W, ci, k=3, pmask=0):
    """dx = adjoint of x -> conv3d(x, W) applied to dy."""
    co = W.shape[0]
    offs = tap_offsets(k)
    Wr = W.reshape(co, len(offs), ci)
    dx = np.zeros(dy.shape[:4] + (ci,))
    for t, (dz, dyo, dxo) in enumerate(offs):
        dx += shift(np.einsum("ndhwo,oc->ndhwc", dy, Wr[:, t, :]), -dz, -dyo, -dxo, pmask)
    return dx


def conv3d_bwd_weight(x, dy, k=3, pmask=0):
    """dW[o, t*ci + c] = sum_p dy[p, o] x[p + off(t), c];  db[o] = sum_p dy[p, o]."""
    offs = tap_offsets(k)
    ci = x.shape[-1]
    co = dy.shape[-1]
    dW = np.zeros((co, len(offs), ci))
    for t, (dz, dyo, dxo) in enumerate(offs):
        dW[:, t, :] = np.einsum("ndhwo,ndhwc->oc", dy, shift(x, dz, dyo, dxo, pmask))
    return dW.reshape(co, -1), dy.sum(axis=(0, 1, 2, 3))


def pool2(x):
    n, d, h, w, c = x.shape
    return x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def pool2_bwd(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_bwd(dy):
    n, d, h, w, c = dy.shape
    return dy.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def mse(out, target):
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(w, g, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
