"""FP64 reference of the surrogate U-Net (forward, loss, gradients), composed
from the layer definitions in conv_ref.py.

TEST INFRASTRUCTURE ONLY.  The GPU network stores activations and gradient
operands in BF16; with bf16=True this reference rounds to BF16 (round to
nearest even) at exactly those points, so the two differ only by FP32-versus-
FP64 accumulation.

Architecture (widths 16-32-64-128, 3x3x3 ReLU convolutions, 2x2x2 average
pooling, nearest upsampling, skip connections by channel concatenation with
the upsampled path first, 1x1x1 head added to the input fields).
"""
from __future__ import annotations

import numpy as np

from . import conv_ref as R

ENC = [("e1a", "e1b"), ("e2a", "e2b"), ("e3a", "e3b"), ("e4a", "e4b")]
DEC = [("d3a", "d3b"), ("d2a", "d2b"), ("d1a", "d1b")]


def bf16(a):
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, x_fields, pmask, round_bf16=True):
    """params: {name: (W[co, k^3 ci], b[co])} (FP32 masters); x_fields:
    (n, d, h, w, 4).  Returns (out, cache)."""
    rb = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W = {k: (rb(w), np.asarray(b, dtype=np.float64)) for k, (w, b) in params.items()}
    n, d, h, w, _ = x_fields.shape
    x_in = np.zeros((n, d, h, w, 8))
    x_in[..., :4] = x_fields
    x_in = rb(x_in)
    cache = {"x_in": x_in}

    def conv(name, x, relu=True):
        y = R.conv3d(x, W[name][0], W[name][1], k=3, pmask=pmask)
        if relu:
            y = R.relu(y)
        return rb(y)

    skips = []
    h_ = x_in
    for lvl, (a, b) in enumerate(ENC):
        ya = conv(a, h_)
        yb = conv(b, ya)
        cache[a], cache[b] = ya, yb
        if lvl < 3:
            skips.append(yb)
            h_ = rb(R.pool2(yb))
            cache["p%d" % (lvl + 1)] = h_
        else:
            h_ = yb
    for (a, b), skip in zip(DEC, reversed(skips)):
        cat = np.concatenate([R.up2(h_), skip], axis=-1)
        cache["cat_" + a] = cat
        ya = conv(a, cat)
        yb = conv(b, ya)
        cache[a], cache[b] = ya, yb
        h_ = yb
    out = np.asarray(x_fields, dtype=np.float32).astype(np.float64) + R.conv3d(h_, W["head"][0], W["head"][1], k=1)
    cache["W"] = W
    return out, cache


def backward(cache, gout, pmask, round_bf16=True):
    """Gradients of a loss with output gradient gout (FP32-like values);
    returns {name: (dW, db)}."""
    rb = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W = cache["W"]
    grads = {}

    def back(name, x, y, gy, need_dx=True, k=3):
        dyb = rb(gy * (y > 0)) if name != "head" else rb(gy)
        grads[name] = R.conv3d_bwd_weight(x, dyb, k=k, pmask=pmask)
        if need_dx:
            return R.conv3d_bwd_data(dyb, W[name][0], x.shape[-1], k=k, pmask=pmask)
        return None

    g = back("head", cache["d1b"], None, gout, k=1)
    gskip = {}
    for (a, b), lvl in zip(reversed(DEC), (0, 1, 2)):       # d1 (skip from e1b), d2, d3
        g = back(b, cache[a], cache[b], g)
        cat = cache["cat_" + a]
        gcat = back(a, cat, cache[a], g)
        cu = cat.shape[-1] - cache[ENC[lvl][1]].shape[-1]
        gskip[lvl] = gcat[..., cu:]
        g = R.up2_bwd(gcat[..., :cu])
    for lvl in (3, 2, 1, 0):
        a, b = ENC[lvl]
        if lvl < 3:
            g = gskip[lvl] + R.pool2_bwd(g)
        g = back(b, cache[a], cache[b], g)
        x = cache["x_in"] if lvl == 0 else cache["p%d" % lvl]
        g = back(a, x, cache[a], g, need_dx=lvl > 0)
    return grads
