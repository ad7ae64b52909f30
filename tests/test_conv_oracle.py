"""Pins of the FP64 reference of the surrogate's layers (oracle/conv_ref.py)
against library primitives (scipy correlation), delta kernels, adjoint
identities and finite differences."""
import numpy as np
import pytest
from scipy import ndimage, signal

from oracle import conv_ref as R


def rnd(*shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("pmask", [0, 7, 5])
def test_conv_matches_scipy_correlation(pmask):
    x = rnd(2, 5, 6, 7, 3, seed=1)
    W = rnd(4, 27 * 3, seed=2)
    b = rnd(4, seed=3)
    y = R.conv3d(x, W, b, k=3, pmask=pmask)
    Wr = W.reshape(4, 3, 3, 3, 3)           # o, dz, dy, dx, c
    for n in range(2):
        for o in range(4):
            acc = np.full(x.shape[1:4], b[o])
            for c in range(3):
                ker = Wr[o, :, :, :, c]
                if pmask == 0:
                    acc += signal.correlate(x[n, ..., c], ker, mode="same")
                elif pmask == 7:
                    acc += ndimage.correlate(x[n, ..., c], ker, mode="wrap")
                else:   # periodic x and z, zero y: pad y with zeros, wrap the others
                    xp = np.pad(x[n, ..., c], ((0, 0), (1, 1), (0, 0)))
                    acc += ndimage.correlate(xp, ker, mode="wrap")[:, 1:-1, :]
            assert np.allclose(y[n, ..., o], acc, atol=1e-12)


def test_delta_kernel_is_a_shift():
    x = rnd(1, 4, 5, 6, 2, seed=4)
    for t, (dz, dy, dx) in enumerate(R.tap_offsets(3)):
        W = np.zeros((3, 27 * 2))
        W[2, t * 2 + 1] = 1.0
        y = R.conv3d(x, W, k=3, pmask=0)
        want = np.zeros(x.shape[:4])
        for z in range(4):
            for yy in range(5):
                for xx in range(6):
                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                    if 0 <= zz < 4 and 0 <= y2 < 5 and 0 <= x2 < 6:
                        want[0, z, yy, xx] = x[0, zz, y2, x2, 1]
        assert np.array_equal(y[..., 2], want)
        assert np.abs(y[..., :2]).max() == 0.0


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("pmask", [0, 3, 7])
def test_adjoint_identities(k, pmask):
    """<conv(x, W), dy> = <x, dx(dy)> = <W, dW(x, dy)>: the data and weight
    gradients are the adjoints of the convolution."""
    x = rnd(2, 4, 6, 8, 5, seed=5)
    W = rnd(3, k ** 3 * 5, seed=6)
    dy = rnd(2, 4, 6, 8, 3, seed=7)
    lhs = np.sum(R.conv3d(x, W, k=k, pmask=pmask) * dy)
    dx = R.conv3d_bwd_data(dy, W, 5, k=k, pmask=pmask)
    dW, db = R.conv3d_bwd_weight(x, dy, k=k, pmask=pmask)
    assert abs(lhs - np.sum(x * dx)) < 1e-10 * abs(lhs) + 1e-10
    assert abs(lhs - np.sum(W * dW)) < 1e-10 * abs(lhs) + 1e-10
    assert np.allclose(db, dy.sum(axis=(0, 1, 2, 3)))


def test_pool_and_upsample_adjoints():
    x = rnd(2, 4, 6, 8, 3, seed=8)
    y = rnd(2, 2, 3, 4, 3, seed=9)
    assert abs(np.sum(R.pool2(x) * y) - np.sum(x * R.pool2_bwd(y))) < 1e-12
    assert abs(np.sum(R.up2(y) * x) - np.sum(y * R.up2_bwd(x))) < 1e-12
    assert np.allclose(R.pool2(R.up2(y)), y)


def test_mse_gradient_finite_difference():
    out = rnd(1, 2, 3, 4, 2, seed=10)
    tgt = rnd(1, 2, 3, 4, 2, seed=11)
    loss, g = R.mse(out, tgt)
    e = np.zeros_like(out)
    e[0, 1, 2, 3, 1] = 1e-6
    fd = (R.mse(out + e, tgt)[0] - R.mse(out - e, tgt)[0]) / 2e-6
    assert abs(fd - g[0, 1, 2, 3, 1]) < 1e-8


def test_adam_first_step():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    w1, m, v = R.adam(w, g, np.zeros(3), np.zeros(3), lr=0.01, b1=0.9, b2=0.999, eps=1e-8, step=1)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("pmask", [0, 5, 7])
def test_pointwise_convolution_matches_the_whole_layer(pmask):
    """conv3d_at (positions one by one, used for layers too large for the
    whole-layer reference) equals conv3d, including positions on every face."""
    rng = np.random.default_rng(3 + pmask)
    x = rng.standard_normal((2, 4, 5, 6, 3))
    W = rng.standard_normal((4, 27 * 3))
    b = rng.standard_normal(4)
    full = R.conv3d(x, W, b, k=3, pmask=pmask)
    pts = np.array([(0, 0, 0, 0), (1, 3, 4, 5), (0, 2, 0, 5), (1, 0, 4, 0), (1, 2, 2, 3)])
    got = R.conv3d_at(x, W, pts, b, k=3, pmask=pmask)
    want = np.array([full[b_, z, y, xx] for b_, z, y, xx in pts])
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)
