"""Pin of the U-Net reference's gradients (oracle/unet_ref.py) against central
finite differences of its own FP64 forward pass (no BF16 rounding)."""
import numpy as np

from oracle import conv_ref as R
from oracle import unet_ref as U


def make_params(rng, scale=0.3):
    spec = {"e1a": (8, 16), "e1b": (16, 16), "e2a": (16, 32), "e2b": (32, 32), "e3a": (32, 64), "e3b": (64, 64),
            "e4a": (64, 128), "e4b": (128, 128), "d3a": (192, 64), "d3b": (64, 64), "d2a": (96, 32),
            "d2b": (32, 32), "d1a": (48, 16), "d1b": (16, 16)}
    p = {k: (rng.standard_normal((co, 27 * ci)) * scale / np.sqrt(27 * ci) * 1.4, rng.standard_normal(co) * 0.05)
         for k, (ci, co) in spec.items()}
    p["head"] = (rng.standard_normal((4, 16)) * 0.2, rng.standard_normal(4) * 0.1)
    return p


def test_unet_reference_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    params = make_params(rng)
    x = rng.standard_normal((1, 8, 8, 8, 4))
    tgt = rng.standard_normal((1, 8, 8, 8, 4))
    out, cache = U.forward(params, x, pmask=3, round_bf16=False)
    loss, gout = R.mse(out, tgt)
    grads = U.backward(cache, gout, pmask=3, round_bf16=False)

    def L(p):
        return R.mse(U.forward(p, x, pmask=3, round_bf16=False)[0], tgt)[0]

    for name, idx in (("head", (2, 5)), ("d1b", (3, 100)), ("e1a", (7, 40)), ("e4b", (100, 2000)),
                      ("d3a", (10, 3000)), ("e2b", (5, 800))):
        W, b = params[name]
        h = 1e-6
        Wp = W.copy(); Wp[idx] += h
        Wm = W.copy(); Wm[idx] -= h
        fd = (L(dict(params, **{name: (Wp, b)})) - L(dict(params, **{name: (Wm, b)}))) / (2 * h)
        assert abs(fd - grads[name][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, fd, grads[name][0][idx])
        bp = b.copy(); bp[idx[0] % b.size] += h
        bm = b.copy(); bm[idx[0] % b.size] -= h
        fdb = (L(dict(params, **{name: (W, bp)})) - L(dict(params, **{name: (W, bm)}))) / (2 * h)
        assert abs(fdb - grads[name][1][idx[0] % b.size]) <= 1e-6 * max(1.0, abs(fdb)), name
