"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/lbcg.h declares, and rejects invalid arguments
before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1904_03618_amd import lbcg as B
from paper_1904_03618_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "lbcg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbcg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.load()
    names = header_functions()
    assert {"lbcg_init", "lbcg_step", "lbcg_moments", "lbcg_free"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTS)


def test_surrogate_library_exports_every_declared_symbol():
    from paper_1904_03618_amd import surrogate as S
    txt = open(os.path.join(ROOT, "include", "lbcg_surrogate.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(sg_[a-z0-9_]+)\s*\(", txt))
    L = B.load()
    for n in names:
        assert hasattr(L, n), n
    assert names == set(S.SG_EXPORTS)


def test_surrogate_entry_points_reject_mismatched_views():
    """Shape and layout checks run on the host before any launch (the view
    pointers here are host memory and are never dereferenced)."""
    from paper_1904_03618_amd import surrogate as S
    L = S.lib()
    buf = np.zeros(1 << 16, dtype=np.float32)
    p = buf.ctypes.data

    def v(n, d, h, w, ctot, coff=0, c=None):
        return C.byref(S.sg_view(p, n, d, h, w, ctot, coff, ctot - coff if c is None else c, 0))

    EINVAL = -1
    # pooling and upsampling: the coarse side must be half the fine side, same channels
    assert L.sg_pool2_fwd(v(1, 4, 4, 4, 8), v(1, 2, 2, 3, 8), None) == EINVAL
    assert L.sg_up2_fwd(v(1, 2, 2, 2, 8), v(1, 4, 4, 4, 16), None) == EINVAL
    # upsampling into a concatenation: y's channels = x's + skip's, skip at y's positions
    assert L.sg_up2_cat_fwd(v(1, 2, 2, 2, 16), v(1, 4, 4, 4, 8), v(1, 4, 4, 4, 32), None) == EINVAL
    assert L.sg_up2_cat_fwd(v(1, 2, 2, 2, 16), v(1, 4, 4, 2, 8), v(1, 4, 4, 4, 24), None) == EINVAL
    assert L.sg_up2_cat_fwd(v(1, 2, 2, 2, 16), v(1, 4, 4, 4, 8), v(1, 4, 4, 3, 24), None) == EINVAL
    assert L.sg_up2_cat_fwd(v(1, 2, 2, 2, 12), v(1, 4, 4, 4, 12), v(1, 4, 4, 4, 24), None) == EINVAL
    # convolution: output channels a multiple of 16, kernel 1 or 3, an output view
    assert L.sg_conv3d_fwd(v(1, 4, 4, 4, 8), p, None, 24, 3, 0, 0, v(1, 4, 4, 4, 24), None, 0, None) == EINVAL
    assert L.sg_conv3d_fwd(v(1, 4, 4, 4, 8), p, None, 16, 5, 0, 0, v(1, 4, 4, 4, 16), None, 0, None) == EINVAL
    assert L.sg_conv3d_fwd(v(1, 4, 4, 4, 8), p, None, 16, 3, 0, 0, None, None, 0, None) == EINVAL
    # no-allocation weight gradient: views checked as for the workspace form,
    # and a problem whose partial sums exceed the library's scratch is refused
    # before anything is launched
    assert L.sg_conv3d_bwd_weight_noalloc(v(1, 4, 4, 4, 8), v(1, 4, 4, 2, 16), 3, 0, p, p, None) == EINVAL
    big = S.sg_view(p, 8, 64, 64, 64, 256, 0, 256, 0)
    assert L.sg_conv3d_bwd_weight_ws(C.byref(big), 256, 3) > (96 << 20)
    assert L.sg_conv3d_bwd_weight_noalloc(C.byref(big), C.byref(big), 3, 0, p, p, None) == EINVAL


def test_struct_layout_matches_header():
    # 6 ints + 10 doubles (5 pairs) + 5 doubles + 7 doubles + 2 ints + 6 doubles (wall velocities)
    assert C.sizeof(B.lbcg_case) == 6 * 4 + 10 * 8 + 5 * 8 + 7 * 8 + 2 * 4 + 6 * 8
    assert C.sizeof(B.lbcg_fields) == 5 * 8 + 8
    assert C.sizeof(B.lbcg_options) == 32


def _init_rc(p, fl=None, opt=None, n=1):
    L = B.load()
    if fl is None:
        N = p["nx"] * p["ny"] * p["nz"]
        fl = {k: np.zeros(N) for k in ("rhoR", "rhoB", "ux", "uy", "uz")}
    cs = (B.lbcg_case * n)(*[B.pack_case(p)] * n)
    fs = (B.lbcg_fields * n)()
    keep = [np.ascontiguousarray(fl[k], dtype=np.float64) for k in ("rhoR", "rhoB", "ux", "uy", "uz")]
    for i in range(n):
        fs[i].rhoR, fs[i].rhoB, fs[i].ux, fs[i].uy, fs[i].uz = [a.ctypes.data for a in keep]
    h = C.c_void_p()
    o = opt if opt is not None else B.lbcg_options(0, 0, 0, 0, 0, 0, 0, 0)
    rc = L.lbcg_init(cs, n, fs, C.byref(o), None, C.byref(h))
    return rc, h.value


@pytest.mark.parametrize("change,frag", [
    (dict(nx=0), "dimensions"),
    (dict(bc=(1, 0, 1)), "one wall axis"),
    (dict(alpha=(1.0, 0.7)), "alpha"),
    (dict(tau_v=(0.5, 0.7)), "tau_v"),
    (dict(tau_q=0.4), "tau_e"),
    (dict(rho_in=(3.0, 1.1)), "pressure balance"),
    (dict(rho_in=(-1.0, 1.0)), "rho_in"),
    (dict(theta_deg=(0.0, 90.0)), "theta"),
    (dict(improved=2), "improved"),
    (dict(wall_u=((0.01, 0.0, 0.0), (0.0, 0.0, 0.0))), "wall axis"),
    (dict(bc=(0, 0, 1), wall_u=((0.0, 0.0, 0.01), (0.0, 0.0, 0.0))), "tangential"),
])
def test_init_rejects_invalid_parameters(change, frag):
    p, _ = W.paper_fluids_droplet(4, 1.0)
    p = dict(p, **change)
    rc, h = _init_rc(p)
    assert rc == B.LBCG_EINVAL and h is None
    assert frag in B.lbcg_last_error()


def test_init_rejects_bad_options_and_pointers():
    p, _ = W.paper_fluids_droplet(4, 1.0)
    rc, _ = _init_rc(p, opt=B.lbcg_options(7, 0, 0, 0, 0, 0, 0, 0))
    assert rc == B.LBCG_EINVAL and "storage" in B.lbcg_last_error()
    rc, _ = _init_rc(p, opt=B.lbcg_options(0, 0, 96 + 1, 0, 0, 0, 0, 0))
    assert rc == B.LBCG_EINVAL and "block_nodes" in B.lbcg_last_error()
    rc, _ = _init_rc(p, opt=B.lbcg_options(0, 0, 0, 0, 5, 0, 0, 0))
    assert rc == B.LBCG_EINVAL and "kernel" in B.lbcg_last_error()
    rc, _ = _init_rc(p, opt=B.lbcg_options(0, 0, 0, 0, 0, -2, 0, 0))
    assert rc == B.LBCG_EINVAL and "zchunk" in B.lbcg_last_error()
    rc, _ = _init_rc(p, opt=B.lbcg_options(0, 0, 0, 0, 0, 0, -1, 0))
    assert rc == B.LBCG_EINVAL and "graph_steps" in B.lbcg_last_error()
    rc, _ = _init_rc(p, opt=B.lbcg_options(0, 0, 0, 0, 0, 0, 0, 3))
    assert rc == B.LBCG_EINVAL and "level" in B.lbcg_last_error()
    # the compact level format exists only with the fused step
    rc, _ = _init_rc(p, opt=B.lbcg_options(0, 0, 0, 0, B.LBCG_KERNEL_TWOPASS, 0, 0, B.LBCG_LEVEL_COMPACT))
    assert rc == B.LBCG_EINVAL and "compact" in B.lbcg_last_error()
    pw = dict(p, bc=(0, 1, 0))
    rc, _ = _init_rc(pw, opt=B.lbcg_options(0, 0, 0, 0, B.LBCG_KERNEL_AUTO, 0, 0, B.LBCG_LEVEL_COMPACT))
    assert rc == B.LBCG_EINVAL and "compact" in B.lbcg_last_error()
    L = B.load()
    h = C.c_void_p()
    assert L.lbcg_init(None, 1, None, None, None, C.byref(h)) == B.LBCG_EINVAL
    assert L.lbcg_init(None, 1, None, None, None, None) == B.LBCG_EINVAL


def test_calls_on_null_handle_fail_cleanly():
    L = B.load()
    assert L.lbcg_step(None, 1) == B.LBCG_ESTATE
    assert L.lbcg_free(None) == B.LBCG_ESTATE
    assert L.lbcg_moments(None, 0, None, None, None, None, None, None, None) == B.LBCG_ESTATE
    assert L.lbcg_steps_done(None) == -1
    assert L.lbcg_case_nodes(None, 0) == -1
    assert L.lbcg_checkpoint_bytes(None) == -1
    buf = C.create_string_buffer(64)
    assert L.lbcg_checkpoint_save(None, buf, 64) == B.LBCG_ESTATE
    assert L.lbcg_checkpoint_load(None, buf, 64) == B.LBCG_ESTATE


def test_init_rejects_cases_beyond_32_bit_offsets():
    """A case whose arrays would exceed the kernels' 32-bit byte offsets is
    rejected before any field is read (the field pointers here are tiny)."""
    L = B.load()
    p, _ = W.paper_fluids_droplet(4, 1.0)
    p = dict(p, nx=1024, ny=1024, nz=256)              # 2^28 nodes
    tiny = np.zeros(4)
    cs = (B.lbcg_case * 1)(B.pack_case(p))
    fs = (B.lbcg_fields * 1)()
    fs[0].rhoR = fs[0].rhoB = fs[0].ux = fs[0].uy = fs[0].uz = tiny.ctypes.data
    h = C.c_void_p()
    o = B.lbcg_options(0, 0, 0, 0, 0, 0, 0, 0)
    assert L.lbcg_init(cs, 1, fs, C.byref(o), None, C.byref(h)) == B.LBCG_EINVAL
    assert h.value is None and "2^28" in B.lbcg_last_error()


def test_never_issued_handle_is_rejected_without_being_read():
    """A pointer lbcg_init never returned is recognised from the registry of
    live handles, so no call dereferences it."""
    L = B.load()
    bogus = C.c_void_p(0x1000)
    assert L.lbcg_step(bogus, 1) == B.LBCG_ESTATE
    assert L.lbcg_free(bogus) == B.LBCG_ESTATE
    assert L.lbcg_steps_done(bogus) == -1 and L.lbcg_case_nodes(bogus, 0) == -1
    assert L.lbcg_storage_bytes(bogus) == -1 and L.lbcg_checkpoint_bytes(bogus) == -1
    assert L.lbcg_step_kernel(bogus) == -1 and L.lbcg_level_format(bogus) == -1
    assert L.lbcg_zchunk(bogus) == -1
