"""The no-allocation weight gradient (sg_conv3d_bwd_weight_noalloc) against
the workspace form (sg_conv3d_bwd_weight) through the C ABI: two calls in a
row on the library's scratch, the second with a smaller input, each equal bit
for bit to the workspace form on the same operands (same kernels, same
partial-sum plan)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _operands(rng, n, d, h, w, ci, co):
    import torch
    x = torch.tensor(rng.standard_normal((n, d, h, w, ci)).astype(np.float32)).to(torch.bfloat16).cuda()
    dy = torch.tensor(rng.standard_normal((n, d, h, w, co)).astype(np.float32)).to(torch.bfloat16).cuda()
    return x, dy


def test_noalloc_weight_gradient_equals_workspace_form():
    import torch
    from paper_1904_03618_amd import surrogate as S
    L = S.lib()
    rng = np.random.default_rng(2024)
    # the larger call first, then a smaller one that reuses (part of) the scratch
    shapes = [((2, 8, 16, 16), 48, 32, 3, 3), ((1, 4, 4, 16), 16, 16, 3, 0)]
    for (n, d, h, w), ci, co, k, pmask in shapes:
        print("noalloc case", (n, d, h, w), ci, co, k, pmask, flush=True)
        x, dy = _operands(rng, n, d, h, w, ci, co)
        xv, dyv = S.view(x), S.view(dy)
        ws_bytes = int(L.sg_conv3d_bwd_weight_ws(C.byref(dyv), ci, k))
        assert 0 < ws_bytes <= (96 << 20)
        ws = torch.empty(ws_bytes // 4 + 1, dtype=torch.float32, device="cuda")
        K = k ** 3 * ci
        dw_ref = torch.full((co, K), float("nan"), device="cuda")
        db_ref = torch.full((co,), float("nan"), device="cuda")
        dw = torch.full((co, K), float("nan"), device="cuda")
        db = torch.full((co,), float("nan"), device="cuda")
        st = S._stream()
        assert L.sg_conv3d_bwd_weight(C.byref(xv), C.byref(dyv), k, pmask, C.c_void_p(dw_ref.data_ptr()),
                                      C.c_void_p(db_ref.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel() * 4,
                                      st) == 0
        assert L.sg_conv3d_bwd_weight_noalloc(C.byref(xv), C.byref(dyv), k, pmask, C.c_void_p(dw.data_ptr()),
                                              C.c_void_p(db.data_ptr()), st) == 0
        torch.cuda.synchronize()
        a, b = dw.cpu().numpy(), dw_ref.cpu().numpy()
        assert np.isfinite(b).all() and np.isfinite(a).all()
        assert np.array_equal(a, b), float(np.abs(a - b).max())
        assert np.array_equal(db.cpu().numpy(), db_ref.cpu().numpy())
        # and against the definition on a few weights (FP64 sums of the BF16 operands)
        x64 = x.float().cpu().numpy().astype(np.float64)
        dy64 = dy.float().cpu().numpy().astype(np.float64)
        assert np.allclose(db.cpu().numpy(), dy64.sum(axis=(0, 1, 2, 3)), rtol=1e-4, atol=1e-3)
        centre = (k ** 3 // 2) * ci                        # the centre tap: no shift, no padding
        want = np.einsum("ndhwo,ndhwc->oc", dy64, x64)
        got = a[:, centre:centre + ci]
        assert np.abs(got - want).max() <= 1e-4 * max(1.0, float(np.abs(want).max())), float(np.abs(got - want).max())
