"""Learned surrogate: a 4-level 3D convolutional U-Net that predicts the phase
field rho^N and the velocity u a fixed number of LB steps ahead.

Every layer runs in the gfx950 kernels of include/lbcg_surrogate.h (BF16 MFMA
convolutions with FP32 accumulation, their data/weight gradients, pooling,
upsampling, loss, Adam); this module only allocates torch device buffers,
wires the layers together and calls the C ABI.

Network (channels-last, widths 16-32-64-128, 3x3x3 convolutions, ReLU):
    enc1: in(8) -> 16 -> 16 -----------------------------------> cat1[32:48]
    pool, enc2: 16 -> 32 -> 32 ---------------------------> cat2[64:96]
    pool, enc3: 32 -> 64 -> 64 -------------------> cat3[128:192]
    pool, bottleneck: 64 -> 128 -> 128, up -> cat3[0:128]
    dec3: 192 -> 64 -> 64, up -> cat2[0:64]
    dec2: 96 -> 32 -> 32, up -> cat1[0:32]
    dec1: 48 -> 16 -> 16, head 1x1x1: 16 -> 4 added to the input fields.
Inputs are (rho^N, u_x/us, u_y/us, u_z/us) padded with zeros to 8 channels
(us: velocity scale); the head starts at zero, so the untrained network
predicts persistence.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import lbcg as B

WIDTHS = (16, 32, 64, 128)
NF = 4          # rho^N, u_x, u_y, u_z
CIN = 8         # input channels padded for the MFMA K groups


class sg_view(C.Structure):
    _fields_ = [("p", C.c_void_p), ("n", C.c_int32), ("d", C.c_int32), ("h", C.c_int32), ("w", C.c_int32),
                ("ctot", C.c_int32), ("coff", C.c_int32), ("c", C.c_int32), ("reserved", C.c_int32)]


SG_EXPORTS = ("sg_conv3d_fwd", "sg_weight_prep", "sg_conv3d_bwd_weight_ws", "sg_conv3d_bwd_weight",
              "sg_conv3d_bwd_weight_noalloc",
              "sg_relu_bwd_cast", "sg_pool2_fwd", "sg_pool2_bwd", "sg_up2_fwd", "sg_up2_bwd", "sg_up2_cat_fwd", "sg_mse",
              "sg_adam", "sg_pack", "sg_unpack", "sg_lift")

_sl = None


def lib():
    global _sl
    if _sl is None:
        L = B.load()
        V = C.POINTER(sg_view)
        vp, i32, i64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
        sig = {
            "sg_conv3d_fwd": [V, vp, vp, i32, i32, i32, i32, V, V, i32, vp],
            "sg_weight_prep": [vp, i32, i32, i32, vp, vp, i32, i32, vp],
            "sg_conv3d_bwd_weight_ws": [V, i32, i32],
            "sg_conv3d_bwd_weight": [V, V, i32, i32, vp, vp, vp, i64, vp],
            "sg_conv3d_bwd_weight_noalloc": [V, V, i32, i32, vp, vp, vp],
            "sg_relu_bwd_cast": [V, V, V, vp],
            "sg_pool2_fwd": [V, V, vp], "sg_pool2_bwd": [V, V, i32, vp],
            "sg_up2_fwd": [V, V, vp], "sg_up2_bwd": [V, V, i32, vp], "sg_up2_cat_fwd": [V, V, V, vp],
            "sg_mse": [V, V, V, vp, vp],
            "sg_adam": [vp, vp, vp, vp, i64, f32, f32, f32, f32, i64, vp],
            "sg_pack": [vp, i32, i32, i32, i32, i32, i32, i32, vp, V, V, i32, vp],
            "sg_unpack": [V, i32, vp, vp, i32, vp],
            "sg_lift": [vp, i64, vp, vp, f64, f64, f64, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = i64 if name == "sg_conv3d_bwd_weight_ws" else C.c_int
        _sl = L
    return _sl


def _chk(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def view(t, coff=0, c=None):
    """sg_view of a channels-last torch tensor (n, d, h, w, ctot)."""
    n, d, h, w, ctot = t.shape
    return sg_view(t.data_ptr(), n, d, h, w, ctot, coff, ctot - coff if c is None else c, 0)


def vptr(v):
    return C.byref(v) if v is not None else None


class Conv:
    """One convolution layer: FP32 master weights + Adam state, BF16 operand
    copies (forward and flipped transpose for the data gradient)."""

    def __init__(self, name, ci, co, k, relu, rng, zero=False):
        import torch
        self.name, self.ci, self.co, self.k, self.relu = name, ci, co, k, relu
        self.K = k ** 3 * ci
        self.co_pad = (co + 15) // 16 * 16
        self.ci_pad = (ci + 15) // 16 * 16
        self.co8 = (co + 7) // 8 * 8
        std = 0.0 if zero else math.sqrt(2.0 / self.K)
        w = rng.standard_normal((co, self.K)).astype(np.float32) * std
        dev = "cuda"
        self.w = torch.tensor(w, device=dev)
        self.b = torch.zeros(co, device=dev)
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.bias_pad = torch.zeros(self.co_pad, device=dev)
        self.wb = torch.zeros(self.co_pad * self.K, dtype=torch.bfloat16, device=dev)
        self.wt = torch.zeros(self.ci_pad * k ** 3 * self.co8, dtype=torch.bfloat16, device=dev)
        self.prep()

    def prep(self):
        _chk(lib().sg_weight_prep(C.c_void_p(self.w.data_ptr()), self.co, self.ci, self.k,
                                  C.c_void_p(self.wb.data_ptr()), C.c_void_p(self.wt.data_ptr()),
                                  self.co_pad, self.ci_pad, _stream()), "sg_weight_prep")
        self.bias_pad[: self.co].copy_(self.b)

    def params(self):
        return [(self.w, self.gw, self.mw, self.vw), (self.b, self.gb, self.mb, self.vb)]

    def fwd(self, x, y=None, y32=None, accumulate=False, pmask=0):
        _chk(lib().sg_conv3d_fwd(vptr(x), C.c_void_p(self.wb.data_ptr()), C.c_void_p(self.bias_pad.data_ptr()),
                                 self.co_pad, self.k, pmask, int(self.relu), vptr(y), vptr(y32), int(accumulate),
                                 _stream()), f"conv fwd {self.name}")

    def bwd_data(self, dyb, dx32, accumulate=False, pmask=0):
        """dx32 (FP32 view, c = ci) = adjoint convolution of the BF16 view dyb (c = co8)."""
        _chk(lib().sg_conv3d_fwd(vptr(dyb), C.c_void_p(self.wt.data_ptr()), None, self.ci_pad, self.k, pmask, 0,
                                 None, vptr(dx32), int(accumulate), _stream()), f"conv bwd data {self.name}")

    def bwd_weight(self, x, dyb, ws, pmask=0):
        _chk(lib().sg_conv3d_bwd_weight(vptr(x), vptr(dyb), self.k, pmask, C.c_void_p(self.gw.data_ptr()),
                                        C.c_void_p(self.gb.data_ptr()), C.c_void_p(ws.data_ptr()),
                                        ws.numel() * 4, _stream()), f"conv bwd weight {self.name}")


class UNet:
    """The surrogate network with preallocated buffers for one input shape
    (n, d, h, w); d, h, w must be multiples of 8."""

    def __init__(self, shape, seed=0, us=0.02, pmask=3):
        import torch
        n, d, h, w = shape
        assert d % 8 == 0 and h % 8 == 0 and w % 8 == 0
        self.shape, self.us, self.pmask = shape, us, pmask
        rng = np.random.default_rng(seed)
        c1, c2, c3, c4 = WIDTHS
        L = [("e1a", CIN, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2), ("e3a", c2, c3),
             ("e3b", c3, c3), ("e4a", c3, c4), ("e4b", c4, c4), ("d3a", c4 + c3, c3), ("d3b", c3, c3),
             ("d2a", c3 + c2, c2), ("d2b", c2, c2), ("d1a", c2 + c1, c1), ("d1b", c1, c1)]
        self.L = {nm: Conv(nm, ci, co, 3, True, rng) for nm, ci, co in L}
        self.L["head"] = Conv("head", c1, NF, 1, False, rng, zero=True)
        self.layers = list(self.L.values())
        self.nparams = sum(l.w.numel() + l.b.numel() for l in self.layers)
        s = [(n, d >> i, h >> i, w >> i) for i in range(4)]
        bf = torch.bfloat16
        A = lambda lvl, c, dt=bf: torch.zeros(s[lvl] + (c,), dtype=dt, device="cuda")
        self.x_in = A(0, CIN)
        self.x32 = A(0, NF, torch.float32)          # input fields (FP32) for the residual
        self.a1, self.cat1, self.d1a, self.d1b = A(0, c1), A(0, c2 + c1), A(0, c1), A(0, c1)
        # the full-resolution skip output in a buffer of its own: written and
        # pooled contiguously, copied into cat1 by the upsampling that fills the
        # rest of cat1's rows (whole-line writes; the backward reads cat1)
        self.s1 = A(0, c1)
        self.p1, self.a2, self.cat2, self.d2a, self.d2b = A(1, c1), A(1, c2), A(1, c3 + c2), A(1, c2), A(1, c2)
        self.p2, self.a3, self.cat3, self.d3a, self.d3b = A(2, c2), A(2, c3), A(2, c4 + c3), A(2, c3), A(2, c3)
        self.p3, self.a4, self.b4 = A(3, c3), A(3, c4), A(3, c4)
        self.out32 = A(0, NF, torch.float32)
        self.tgt32 = A(0, NF, torch.float32)
        f32 = torch.float32
        G = lambda t: torch.zeros(t.shape, dtype=f32, device="cuda")
        self.g = {k: G(getattr(self, k)) for k in ("a1", "cat1", "d1a", "d1b", "p1", "a2", "cat2", "d2a", "d2b",
                                                   "p2", "a3", "cat3", "d3a", "d3b", "p3", "a4", "b4", "out32")}
        self.dyb = [A(i, WIDTHS[i]) for i in range(4)]
        self.tgt_bf = A(0, CIN)                      # BF16 image of the target (unused)
        self.dyb_head = A(0, 8)
        self.loss = torch.zeros(257, dtype=torch.float64, device="cuda")
        wsz = 0
        for l in self.layers:
            lvl = {"e1": 0, "d1": 0, "he": 0, "e2": 1, "d2": 1, "e3": 2, "d3": 2, "e4": 3}[l.name[:2]]
            dyv = sg_view(1, *s[lvl], l.co8, 0, l.co, 0)      # size query only
            wsz = max(wsz, int(lib().sg_conv3d_bwd_weight_ws(C.byref(dyv), l.ci, l.k)))
        self.ws = torch.zeros(wsz // 4 + 1, dtype=f32, device="cuda")
        self.step_count = 0

    # ------------------------------------------------------------ forward
    def forward(self):
        """x_in / x32 must be filled; result in out32 (FP32, 4 channels)."""
        L, c1, c2, c3, c4, pm = self.L, *WIDTHS, self.pmask
        v = view
        L["e1a"].fwd(v(self.x_in), v(self.a1), pmask=pm)
        L["e1b"].fwd(v(self.a1), v(self.s1), pmask=pm)
        _chk(lib().sg_pool2_fwd(C.byref(v(self.s1)), C.byref(v(self.p1)), _stream()), "pool1")
        L["e2a"].fwd(v(self.p1), v(self.a2), pmask=pm)
        L["e2b"].fwd(v(self.a2), v(self.cat2, c3, c2), pmask=pm)
        _chk(lib().sg_pool2_fwd(C.byref(v(self.cat2, c3, c2)), C.byref(v(self.p2)), _stream()), "pool2")
        L["e3a"].fwd(v(self.p2), v(self.a3), pmask=pm)
        L["e3b"].fwd(v(self.a3), v(self.cat3, c4, c3), pmask=pm)
        _chk(lib().sg_pool2_fwd(C.byref(v(self.cat3, c4, c3)), C.byref(v(self.p3)), _stream()), "pool3")
        L["e4a"].fwd(v(self.p3), v(self.a4), pmask=pm)
        L["e4b"].fwd(v(self.a4), v(self.b4), pmask=pm)
        _chk(lib().sg_up2_fwd(C.byref(v(self.b4)), C.byref(v(self.cat3, 0, c4)), _stream()), "up3")
        L["d3a"].fwd(v(self.cat3), v(self.d3a), pmask=pm)
        L["d3b"].fwd(v(self.d3a), v(self.d3b), pmask=pm)
        _chk(lib().sg_up2_fwd(C.byref(v(self.d3b)), C.byref(v(self.cat2, 0, c3)), _stream()), "up2")
        L["d2a"].fwd(v(self.cat2), v(self.d2a), pmask=pm)
        L["d2b"].fwd(v(self.d2a), v(self.d2b), pmask=pm)
        _chk(lib().sg_up2_cat_fwd(C.byref(v(self.d2b)), C.byref(v(self.s1)), C.byref(v(self.cat1)), _stream()),
             "up1")
        L["d1a"].fwd(v(self.cat1), v(self.d1a), pmask=pm)
        L["d1b"].fwd(v(self.d1a), v(self.d1b), pmask=pm)
        self.out32.copy_(self.x32)
        L["head"].fwd(v(self.d1b), None, v(self.out32), accumulate=True, pmask=pm)

    # ----------------------------------------------------------- backward
    def _conv_back(self, layer, x, y, gy, gx, lvl, gx_accumulate=False):
        """Through ReLU(conv): weight/bias gradients and, if gx, the input gradient."""
        dyv = view(self.dyb[lvl], 0, layer.co)
        _chk(lib().sg_relu_bwd_cast(C.byref(gy), C.byref(y), C.byref(dyv), _stream()), "relu bwd")
        layer.bwd_weight(x, dyv, self.ws, pmask=self.pmask)
        if gx is not None:
            layer.bwd_data(view(self.dyb[lvl], 0, layer.co8), gx, accumulate=gx_accumulate, pmask=self.pmask)

    def backward(self):
        """Gradients of the loss whose output gradient is in g['out32']."""
        L, g, v, (c1, c2, c3, c4) = self.L, self.g, view, WIDTHS
        hd = L["head"]
        gout = v(g["out32"])
        dh = v(self.dyb_head, 0, NF)
        _chk(lib().sg_relu_bwd_cast(C.byref(gout), None, C.byref(dh), _stream()), "head cast")
        hd.bwd_weight(v(self.d1b), dh, self.ws, pmask=self.pmask)
        hd.bwd_data(v(self.dyb_head), v(g["d1b"]), pmask=self.pmask)
        self._conv_back(L["d1b"], v(self.d1a), v(self.d1b), v(g["d1b"]), v(g["d1a"]), 0)
        self._conv_back(L["d1a"], v(self.cat1), v(self.d1a), v(g["d1a"]), v(g["cat1"]), 0)
        _chk(lib().sg_up2_bwd(C.byref(v(g["cat1"], 0, c2)), C.byref(v(g["d2b"])), 0, _stream()), "up1 bwd")
        self._conv_back(L["d2b"], v(self.d2a), v(self.d2b), v(g["d2b"]), v(g["d2a"]), 1)
        self._conv_back(L["d2a"], v(self.cat2), v(self.d2a), v(g["d2a"]), v(g["cat2"]), 1)
        _chk(lib().sg_up2_bwd(C.byref(v(g["cat2"], 0, c3)), C.byref(v(g["d3b"])), 0, _stream()), "up2 bwd")
        self._conv_back(L["d3b"], v(self.d3a), v(self.d3b), v(g["d3b"]), v(g["d3a"]), 2)
        self._conv_back(L["d3a"], v(self.cat3), v(self.d3a), v(g["d3a"]), v(g["cat3"]), 2)
        _chk(lib().sg_up2_bwd(C.byref(v(g["cat3"], 0, c4)), C.byref(v(g["b4"])), 0, _stream()), "up3 bwd")
        self._conv_back(L["e4b"], v(self.a4), v(self.b4), v(g["b4"]), v(g["a4"]), 3)
        self._conv_back(L["e4a"], v(self.p3), v(self.a4), v(g["a4"]), v(g["p3"]), 3)
        _chk(lib().sg_pool2_bwd(C.byref(v(g["p3"])), C.byref(v(g["cat3"], c4, c3)), 1, _stream()), "pool3 bwd")
        self._conv_back(L["e3b"], v(self.a3), v(self.cat3, c4, c3), v(g["cat3"], c4, c3), v(g["a3"]), 2)
        self._conv_back(L["e3a"], v(self.p2), v(self.a3), v(g["a3"]), v(g["p2"]), 2)
        _chk(lib().sg_pool2_bwd(C.byref(v(g["p2"])), C.byref(v(g["cat2"], c3, c2)), 1, _stream()), "pool2 bwd")
        self._conv_back(L["e2b"], v(self.a2), v(self.cat2, c3, c2), v(g["cat2"], c3, c2), v(g["a2"]), 1)
        self._conv_back(L["e2a"], v(self.p1), v(self.a2), v(g["a2"]), v(g["p1"]), 1)
        _chk(lib().sg_pool2_bwd(C.byref(v(g["p1"])), C.byref(v(g["cat1"], c2, c1)), 1, _stream()), "pool1 bwd")
        self._conv_back(L["e1b"], v(self.a1), v(self.cat1, c2, c1), v(g["cat1"], c2, c1), v(g["a1"]), 0)
        self._conv_back(L["e1a"], v(self.x_in), v(self.a1), v(g["a1"]), None, 0)

    def mse(self):
        """Loss of out32 against tgt32 (device double in self.loss[0]) and its gradient."""
        _chk(lib().sg_mse(C.byref(view(self.out32)), C.byref(view(self.tgt32)), C.byref(view(self.g["out32"])),
                          C.c_void_p(self.loss.data_ptr()), _stream()), "mse")

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        for l in self.layers:
            for w, g, m, v in l.params():
                _chk(lib().sg_adam(C.c_void_p(w.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(m.data_ptr()),
                                   C.c_void_p(v.data_ptr()), w.numel(), lr, b1, b2, eps, self.step_count,
                                   _stream()), "adam")
            l.prep()

    # ------------------------------------------------------------- fields
    def _scale(self):
        return (C.c_float * NF)(1.0, *([self.us] * (NF - 1)))

    def pack(self, fields, box, origin=(0, 0, 0), b=0, target=False):
        """fields: CUDA float32 (4, nz*ny*nx) planar (rho^N, u_x, u_y, u_z) of an
        nx*ny*nz box = `box`; the network sees (rho^N, u/us)."""
        nx, ny, nz = box
        bf, f32 = (self.tgt_bf, self.tgt32) if target else (self.x_in, self.x32)
        _chk(lib().sg_pack(C.c_void_p(fields.data_ptr()), NF, nx, ny, nz, *origin, self._scale(), C.byref(view(bf)),
                           C.byref(view(f32)), b, _stream()), "pack")

    def unpack(self, out, b=0):
        """Prediction of batch item b back to physical planar fields (4, nz*ny*nx)."""
        _chk(lib().sg_unpack(C.byref(view(self.out32)), b, self._scale(), C.c_void_p(out.data_ptr()), NF,
                             _stream()), "unpack")

    def state_dict(self):
        return {l.name: (l.w.cpu().numpy(), l.b.cpu().numpy()) for l in self.layers}

    def load_state(self, sd):
        import torch
        for l in self.layers:
            w, b = sd[l.name]
            l.w.copy_(torch.tensor(w))
            l.b.copy_(torch.tensor(b))
            l.prep()


def lift(pred, cs2, rho_prev=None, p_in=None):
    """(4, n) CUDA float32 prediction -> (5, n) CUDA float64 (rho_R, rho_B, u)
    whose phase field is the predicted rho^N and whose pressure is the one of
    the state before the jump (rho_prev = (rho_R, rho_B) FP32) or p_in."""
    import torch
    n = pred.shape[1]
    out = torch.empty((5, n), dtype=torch.float64, device="cuda")
    pr = (C.c_void_p(rho_prev[0].data_ptr()), C.c_void_p(rho_prev[1].data_ptr())) if rho_prev is not None else (None, None)
    _chk(lib().sg_lift(C.c_void_p(pred.data_ptr()), n, *pr, float(cs2[0]), float(cs2[1]),
                       float(p_in if p_in is not None else 0.0), C.c_void_p(out.data_ptr()), _stream()), "lift")
    return out



LEVEL = {"e1": 0, "d1": 0, "he": 0, "e2": 1, "d2": 1, "e3": 2, "d3": 2, "e4": 3}


def flops(net):
    """Algorithmic FLOPs (2 per multiply-add) of one forward pass and of one
    training step (forward, weight gradients, data gradients of every layer
    but the first) of the network at its buffer shape.  The first layer counts
    its NF real input channels, not the zero channels that pad them to CIN."""
    n, d, h, w = net.shape
    fwd = bwd_w = bwd_x = 0
    for l in net.layers:
        lv = LEVEL[l.name[:2]]
        P = n * (d >> lv) * (h >> lv) * (w >> lv)
        ci = NF if l.name == "e1a" else l.ci
        f = 2 * P * l.co * l.k ** 3 * ci
        fwd += f
        bwd_w += f
        if l.name != "e1a":
            bwd_x += f
    return fwd, fwd + bwd_w + bwd_x


def bench_unet(shape, iters=10, train=True, warmup=2):
    """Time the forward pass (and a training step) of the network at `shape`
    with HIP events on the current stream; returns ms and TFLOP/s."""
    import torch
    net = UNet(shape, seed=1, us=0.02, pmask=3)
    n, d, h, w = shape
    g = torch.Generator(device="cuda").manual_seed(3)
    f = 0.1 * torch.randn((4, d * h * w), device="cuda", generator=g)
    for b in range(n):
        net.pack(f, (w, h, d), b=b)
        net.pack(f, (w, h, d), b=b, target=True)
    fl_fwd, fl_train = flops(net)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"shape": list(shape), "params": net.nparams, "forward_gflop": fl_fwd / 1e9}
    for _ in range(warmup):
        net.forward()
    e0.record()
    for _ in range(iters):
        net.forward()
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / iters
    out.update(forward_ms=ms, forward_tflops=fl_fwd / (ms * 1e-3) / 1e12)
    if train:
        for _ in range(warmup):
            net.forward(); net.mse(); net.backward(); net.adam(1e-4)
        e0.record()
        for _ in range(iters):
            net.forward(); net.mse(); net.backward(); net.adam(1e-4)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / iters
        out.update(train_gflop=fl_train / 1e9, train_ms=ms, train_tflops=fl_train / (ms * 1e-3) / 1e12)
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Time the surrogate network's forward pass and training step")
    ap.add_argument("--shape", default="1,512,128,128", help="batch,depth,height,width")
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--no-train", action="store_true")
    a = ap.parse_args()
    print(json.dumps(bench_unet(tuple(int(v) for v in a.shape.split(",")), a.iters, not a.no_train)), flush=True)
