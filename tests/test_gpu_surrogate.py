"""The surrogate's gfx950 kernels (BF16 MFMA convolutions and their
gradients, element-wise layers, the whole U-Net's gradients) against the FP64
references in oracle/conv_ref.py and oracle/unet_ref.py.  Inputs are BF16
values, so the references see exactly the operands the kernels see; the
remaining difference is FP32 accumulation order."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def bft(a):
    """numpy -> CUDA bfloat16 tensor, and the exact values back as float64."""
    import torch
    t = torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()
    return t, t.float().cpu().numpy().astype(np.float64)


def f32t(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32)).cuda()


def close(got, want, rtol=2e-5):
    scale = max(1e-30, float(np.abs(want).max()))
    err = float(np.abs(got - want).max()) / scale
    return err <= rtol, err


@pytest.mark.parametrize("k,pmask,shape,ctot,coff,ci,co", [
    (3, 0, (1, 4, 6, 16), 8, 0, 8, 16),
    (3, 3, (2, 8, 8, 8), 48, 0, 48, 16),
    (3, 7, (1, 4, 8, 8), 48, 32, 16, 32),
    (1, 0, (1, 5, 7, 9), 16, 0, 16, 4),
    (3, 5, (1, 8, 4, 8), 64, 0, 64, 128),
    # extents that are multiples of the 16 x 4 x 4 brick (LDS-staged halo path)
    (3, 0, (1, 4, 4, 16), 8, 0, 8, 16),
    (3, 7, (2, 8, 4, 32), 64, 16, 48, 32),
    (3, 3, (1, 4, 8, 16), 192, 0, 192, 64),
    (3, 6, (1, 8, 8, 16), 16, 0, 16, 16),
    # 24 mod 32 input channels on bricks of one plane per wave (16-channel chunks)
    (3, 0, (1, 4, 4, 16), 24, 0, 24, 16),
    (3, 5, (1, 4, 4, 16), 64, 8, 56, 32),
])
def test_conv_forward_data_and_weight_gradients(k, pmask, shape, ctot, coff, ci, co):
    import torch
    from oracle import conv_ref as R
    from paper_1904_03618_amd import surrogate as S
    rng = np.random.default_rng(ci * 7 + co)
    n, d, h, w = shape
    xt, _ = bft(rng.standard_normal((n, d, h, w, ctot)))
    x64 = xt.float().cpu().numpy().astype(np.float64)[..., coff:coff + ci]
    layer = S.Conv("t", ci, co, k, False, rng)
    layer.b.copy_(torch.tensor(rng.standard_normal(co).astype(np.float32)))
    layer.prep()
    W64 = layer.w.to(torch.bfloat16).float().cpu().numpy().astype(np.float64)
    b64 = layer.b.cpu().numpy().astype(np.float64)
    y32 = torch.zeros((n, d, h, w, co), device="cuda")
    layer.fwd(S.view(xt, coff, ci), None, S.view(y32), pmask=pmask)
    ok, err = close(y32.cpu().numpy(), R.conv3d(x64, W64, b64, k=k, pmask=pmask))
    print("fwd", k, pmask, ci, co, err, flush=True)
    assert ok, err
    # data gradient: adjoint convolution with the flipped transposed weights
    co8 = layer.co8
    dyt, dy64 = bft(np.concatenate([rng.standard_normal((n, d, h, w, co)), np.zeros((n, d, h, w, co8 - co))], -1))
    dx32 = torch.zeros((n, d, h, w, ci), device="cuda")
    layer.bwd_data(S.view(dyt), S.view(dx32), pmask=pmask)
    ok, err = close(dx32.cpu().numpy(), R.conv3d_bwd_data(dy64[..., :co], W64, ci, k=k, pmask=pmask))
    print("bwd data", err, flush=True)
    assert ok, err
    # weight and bias gradients
    ws = torch.zeros(int(S.lib().sg_conv3d_bwd_weight_ws(C.byref(S.view(dyt, 0, co)), ci, k)) // 4 + 1, device="cuda")
    layer.bwd_weight(S.view(xt, coff, ci), S.view(dyt, 0, co), ws, pmask=pmask)
    dW, db = R.conv3d_bwd_weight(x64, dy64[..., :co], k=k, pmask=pmask)
    ok, err = close(layer.gw.cpu().numpy(), dW)
    ok2, err2 = close(layer.gb.cpu().numpy(), db)
    print("bwd weight", err, err2, flush=True)
    assert ok and ok2, (err, err2)


@pytest.mark.parametrize("pmask", [3, 0])
def test_large_layer_two_plane_bricks(pmask):
    """A layer large enough for the two-plane, 32-channel brick (1 x 64 x 64 x
    128 positions, 32 -> 64 channels: 2048 workgroups, above the 512 that
    select it), checked at
    sampled positions (faces and corners included) against the convolution's
    definition evaluated there."""
    import torch
    from oracle import conv_ref as R
    from paper_1904_03618_amd import surrogate as S
    rng = np.random.default_rng(91 + pmask)
    n, d, h, w, ci, co = 1, 64, 64, 128, 32, 64
    xt, x64 = bft(rng.standard_normal((n, d, h, w, ci)))
    layer = S.Conv("big", ci, co, 3, False, rng)
    layer.b.copy_(torch.tensor(rng.standard_normal(co).astype(np.float32)))
    layer.prep()
    W64 = layer.w.to(torch.bfloat16).float().cpu().numpy().astype(np.float64)
    b64 = layer.b.cpu().numpy().astype(np.float64)
    y32 = torch.zeros((n, d, h, w, co), device="cuda")
    layer.fwd(S.view(xt), None, S.view(y32), pmask=pmask)
    pts = np.stack([rng.integers(0, s_, 300) for s_ in (n, d, h, w)], axis=1)
    pts = np.concatenate([pts, [(0, 0, 0, 0), (0, d - 1, h - 1, w - 1), (0, 0, h - 1, 0), (0, d - 1, 0, w - 1)]])
    got = y32.cpu().numpy()[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]]
    ok, err = close(got, R.conv3d_at(x64, W64, pts, b64, k=3, pmask=pmask))
    print("large layer", pmask, err, flush=True)
    assert ok, err


def test_elementwise_layers():
    import torch
    from oracle import conv_ref as R
    from paper_1904_03618_amd import surrogate as S
    L = S.lib()
    st = S._stream()
    rng = np.random.default_rng(5)
    xt, x64 = bft(rng.standard_normal((2, 4, 6, 8, 8)))
    p = torch.zeros((2, 2, 3, 4, 8), dtype=torch.bfloat16, device="cuda")
    assert L.sg_pool2_fwd(C.byref(S.view(xt)), C.byref(S.view(p)), st) == 0
    assert close(p.float().cpu().numpy(), R.pool2(x64), 4e-3)[0]     # BF16 result
    up = torch.zeros_like(xt)
    assert L.sg_up2_fwd(C.byref(S.view(p)), C.byref(S.view(up)), st) == 0
    assert np.array_equal(up.float().cpu().numpy(), R.up2(p.float().cpu().numpy()))
    # upsampling into a concatenation: [up2(coarse) | skip] per position, with
    # the destination a channel slice of a wider buffer
    coarse, _ = bft(rng.standard_normal((2, 2, 3, 4, 16)))
    skip, _ = bft(rng.standard_normal((2, 4, 6, 8, 8)))
    wide = torch.full((2, 4, 6, 8, 40), 7.0, dtype=torch.bfloat16, device="cuda")
    assert L.sg_up2_cat_fwd(C.byref(S.view(coarse)), C.byref(S.view(skip)), C.byref(S.view(wide, 8, 24)), st) == 0
    w = wide.float().cpu().numpy()
    assert np.array_equal(w[..., 8:24], R.up2(coarse.float().cpu().numpy()))
    assert np.array_equal(w[..., 24:32], skip.float().cpu().numpy())
    assert (w[..., :8] == 7.0).all() and (w[..., 32:] == 7.0).all()
    assert L.sg_up2_cat_fwd(C.byref(S.view(coarse)), C.byref(S.view(skip)), C.byref(S.view(wide, 0, 32)), st) != 0
    g = f32t(rng.standard_normal((2, 2, 3, 4, 8)))
    gx = f32t(np.ones((2, 4, 6, 8, 8)))
    assert L.sg_pool2_bwd(C.byref(S.view(g)), C.byref(S.view(gx)), 1, st) == 0
    assert close(gx.cpu().numpy(), 1 + R.pool2_bwd(g.cpu().numpy().astype(np.float64)))[0]
    gg = f32t(rng.standard_normal((2, 4, 6, 8, 8)))
    gp = torch.zeros((2, 2, 3, 4, 8), device="cuda")
    assert L.sg_up2_bwd(C.byref(S.view(gg)), C.byref(S.view(gp)), 0, st) == 0
    assert close(gp.cpu().numpy(), R.up2_bwd(gg.cpu().numpy().astype(np.float64)))[0]
    dyb = torch.zeros_like(xt)
    assert L.sg_relu_bwd_cast(C.byref(S.view(gg)), C.byref(S.view(xt)), C.byref(S.view(dyb)), st) == 0
    want = gg.cpu().numpy() * (x64 > 0)
    assert np.array_equal(dyb.float().cpu().numpy(), torch.tensor(want.astype(np.float32)).to(torch.bfloat16).float().numpy())
    out = f32t(rng.standard_normal((1, 2, 4, 8, 4)))
    tgt = f32t(rng.standard_normal((1, 2, 4, 8, 4)))
    grad = torch.zeros_like(out)
    loss = torch.zeros(257, dtype=torch.float64, device="cuda")
    assert L.sg_mse(C.byref(S.view(out)), C.byref(S.view(tgt)), C.byref(S.view(grad)), C.c_void_p(loss.data_ptr()), st) == 0
    l64, g64 = R.mse(out.cpu().numpy().astype(np.float64), tgt.cpu().numpy().astype(np.float64))
    assert abs(loss[0].item() - l64) < 1e-6 * l64 and close(grad.cpu().numpy(), g64, 1e-6)[0]
    w = f32t(rng.standard_normal(1000))
    gw = f32t(rng.standard_normal(1000))
    m = torch.zeros(1000, device="cuda"); v = torch.zeros(1000, device="cuda")
    wn, mn, vn = w.cpu().numpy().astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in (1, 2, 3):
        assert L.sg_adam(C.c_void_p(w.data_ptr()), C.c_void_p(gw.data_ptr()), C.c_void_p(m.data_ptr()),
                         C.c_void_p(v.data_ptr()), 1000, 1e-2, 0.9, 0.999, 1e-8, step, st) == 0
        wn, mn, vn = R.adam(wn, gw.cpu().numpy().astype(np.float64), mn, vn, 1e-2, 0.9, 0.999, 1e-8, step)
    assert close(w.cpu().numpy(), wn, 1e-6)[0]


@pytest.mark.parametrize("pmask", [3, 0])
def test_unet_loss_and_gradients_match_oracle(pmask):
    """One forward/backward of the whole network on an 8^3 box (batch 2):
    loss and every layer's weight and bias gradients, element by element,
    against the FP64 reference that rounds to BF16 where the kernels store
    BF16 (the remaining difference is FP32 accumulation order, which can flip
    a BF16 rounding of an intermediate operand by 2^-8 relative)."""
    import torch
    from oracle import conv_ref as R
    from oracle import unet_ref as U
    from paper_1904_03618_amd import surrogate as S
    rng = np.random.default_rng(11)
    net = S.UNet((2, 8, 8, 8), seed=4, pmask=pmask, us=1.0)
    for l in net.layers:                          # a non-trivial head and biases
        l.w.mul_(1.0 if l.name != "head" else 0.0).add_(
            torch.tensor(rng.standard_normal(l.w.shape).astype(np.float32) * (0.2 if l.name == "head" else 0.0)).cuda())
        l.b.copy_(torch.tensor(rng.standard_normal(l.co).astype(np.float32) * 0.05))
        l.prep()
    x = rng.standard_normal((2, 8, 8, 8, 4)).astype(np.float32)
    t = rng.standard_normal((2, 8, 8, 8, 4)).astype(np.float32)
    f = torch.tensor(np.moveaxis(x, -1, 1).reshape(2, 4, -1)).cuda()
    ft = torch.tensor(np.moveaxis(t, -1, 1).reshape(2, 4, -1)).cuda()
    for b in range(2):
        net.pack(f[b].contiguous(), (8, 8, 8), b=b)
        net.pack(ft[b].contiguous(), (8, 8, 8), b=b, target=True)
    net.forward()
    net.mse()
    net.backward()
    torch.cuda.synchronize()
    params = {l.name: (l.w.cpu().numpy(), l.b.cpu().numpy()) for l in net.layers}
    out, cache = U.forward(params, x.astype(np.float64), pmask=pmask, round_bf16=True)
    loss, gout = R.mse(out, t.astype(np.float64))
    grads = U.backward(cache, gout, pmask=pmask, round_bf16=True)
    ok, err = close(net.out32.cpu().numpy(), out, 1e-3)
    print("out", err, "loss", net.loss[0].item(), loss, flush=True)
    assert ok, err
    assert abs(net.loss[0].item() - loss) < 1e-3 * loss
    # per layer, element by element: the largest weight (bias) gradient error
    # relative to the largest weight (bias) gradient of that layer
    for l in net.layers:
        gW, gb = grads[l.name]
        a, b = l.gw.cpu().numpy().astype(np.float64), gW
        ew = float(np.abs(a - b).max()) / max(1e-30, float(np.abs(b).max()))
        ab = l.gb.cpu().numpy().astype(np.float64)
        eb = float(np.abs(ab - gb).max()) / max(1e-30, float(np.abs(gb).max()))
        print(l.name, "dW max-abs rel %.2e  db max-abs rel %.2e" % (ew, eb), flush=True)
        assert ew < 1e-2 and eb < 1e-2, l.name


def test_unet_training_reduces_loss():
    """A few Adam steps on a fixed pair lower the loss (the network learns a
    smooth map from the inputs)."""
    import torch
    from paper_1904_03618_amd import surrogate as S
    rng = np.random.default_rng(2)
    net = S.UNet((1, 16, 16, 16), seed=1, pmask=7, us=1.0)
    z, y, x = np.meshgrid(*[np.arange(16)] * 3, indexing="ij")
    base = np.stack([np.sin(2 * np.pi * (x + 2 * y) / 16), np.cos(2 * np.pi * z / 16), 0 * x, 0.5 * np.sin(2 * np.pi * y / 16)])
    tgt = np.roll(base, 1, axis=3) * 0.9
    net.pack(torch.tensor(base.reshape(4, -1).astype(np.float32)).cuda(), (16, 16, 16))
    net.pack(torch.tensor(tgt.reshape(4, -1).astype(np.float32)).cuda(), (16, 16, 16), target=True)
    losses = []
    for it in range(30):
        net.forward()
        net.mse()
        losses.append(net.loss[0].item())
        net.backward()
        net.adam(2e-3)
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_lift_matches_oracle():
    """sg_lift against the FP64 lift reference, at the pre-jump pressure and at
    a uniform pressure; velocities copied; EINVAL on mismatched pointers."""
    import torch
    from oracle import lift_ref as LR
    from paper_1904_03618_amd import surrogate as S
    rng = np.random.default_rng(8)
    n = 70001
    pred = f32t(np.concatenate([rng.uniform(-1.2, 1.2, (1, n)), 0.03 * rng.standard_normal((3, n))]))
    rR = f32t(rng.uniform(0.0, 3.2, n))
    rB = f32t(rng.uniform(0.0, 1.1, n))
    cs2 = (0.05, 0.15)
    out = S.lift(pred, cs2, rho_prev=(rR, rB)).cpu().numpy()
    pv = pred.cpu().numpy().astype(np.float64)
    p = rR.cpu().numpy().astype(np.float64) * cs2[0] + rB.cpu().numpy().astype(np.float64) * cs2[1]
    wR, wB = LR.lift(pv[0], p, *cs2)
    assert close(out[0], wR, 1e-6)[0] and close(out[1], wB, 1e-6)[0]
    assert np.array_equal(out[2:], pv[1:])
    out = S.lift(pred, cs2, p_in=0.15).cpu().numpy()
    wR, wB = LR.lift(pv[0], 0.15, *cs2)
    assert close(out[0], wR, 1e-6)[0] and close(out[1], wB, 1e-6)[0]
    o = torch.empty(5 * n, dtype=torch.float64, device="cuda")
    rc = S.lib().sg_lift(C.c_void_p(pred.data_ptr()), n, C.c_void_p(rR.data_ptr()), None, 0.05, 0.15, 0.15,
                         C.c_void_p(o.data_ptr()), S._stream())
    assert rc != 0
