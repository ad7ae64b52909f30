"""Python binding of the C ABI in include/lbcg.h (argument marshalling only).

The functions carry the names of the C entry points.  Every step of the
method runs in the gfx950 kernels of liblbcg.so; this module only packs
parameters into the C structs, hands torch-allocated device buffers and the
current HIP stream to the library and raises on error codes.  There is no
fallback: if the library is missing or no GPU is present the calls fail.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbcg.so")

LBCG_OK, LBCG_EINVAL, LBCG_ENOMEM, LBCG_EDEVICE, LBCG_EUNSTABLE, LBCG_ESTATE = 0, -1, -2, -3, -4, -5
LBCG_FP32, LBCG_FP16S, LBCG_BF16S = 0, 1, 2
STORAGE = {"fp32": LBCG_FP32, "fp16s": LBCG_FP16S, "bf16s": LBCG_BF16S}

# Every symbol include/lbcg.h declares.
EXPORTS = ("lbcg_init", "lbcg_step", "lbcg_moments", "lbcg_free", "lbcg_last_error",
           "lbcg_steps_done", "lbcg_index_map", "lbcg_get_populations", "lbcg_case_nodes",
           "lbcg_storage_bytes", "lbcg_timing", "lbcg_timing_read", "lbcg_set_fields", "lbcg_checkpoint_bytes",
           "lbcg_checkpoint_save", "lbcg_checkpoint_load", "lbcg_step_kernel", "lbcg_level_format",
           "lbcg_zchunk")


class LbcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbcg error {code}: {msg}")
        self.code = code


class lbcg_case(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("bc", C.c_int32 * 3),
                ("theta_deg", C.c_double * 2), ("rho_in", C.c_double * 2),
                ("alpha", C.c_double * 2), ("tau_v", C.c_double * 2), ("A", C.c_double * 2),
                ("beta", C.c_double), ("delta", C.c_double),
                ("tau_e", C.c_double), ("tau_q", C.c_double), ("tau_pi", C.c_double),
                ("force", C.c_double * 3), ("grav", C.c_double * 3), ("rho_ref", C.c_double),
                ("improved", C.c_int32), ("meq4", C.c_int32),
                ("wall_u", (C.c_double * 3) * 2)]


class lbcg_fields(C.Structure):
    _fields_ = [("rhoR", C.c_void_p), ("rhoB", C.c_void_p), ("ux", C.c_void_p),
                ("uy", C.c_void_p), ("uz", C.c_void_p), ("on_device", C.c_int32),
                ("reserved", C.c_int32)]


class lbcg_options(C.Structure):
    _fields_ = [("storage", C.c_int32), ("diag_every", C.c_int32),
                ("block_nodes", C.c_int32), ("persistent_blocks", C.c_int32),
                ("kernel", C.c_int32), ("zchunk", C.c_int32),
                ("graph_steps", C.c_int32), ("level", C.c_int32)]


LBCG_KERNEL_AUTO, LBCG_KERNEL_TWOPASS, LBCG_KERNEL_FUSED = 0, 1, 2
KERNEL = {"auto": LBCG_KERNEL_AUTO, "twopass": LBCG_KERNEL_TWOPASS, "fused": LBCG_KERNEL_FUSED}
LBCG_LEVEL_AUTO, LBCG_LEVEL_PAIR, LBCG_LEVEL_COMPACT = 0, 1, 2
LEVEL = {"auto": LBCG_LEVEL_AUTO, "pair": LBCG_LEVEL_PAIR, "compact": LBCG_LEVEL_COMPACT}


_lib = None


def load():
    """Load liblbcg.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.lbcg_init.argtypes = [C.POINTER(lbcg_case), i32, C.POINTER(lbcg_fields),
                            C.POINTER(lbcg_options), vp, C.POINTER(vp)]
    L.lbcg_init.restype = C.c_int
    L.lbcg_step.argtypes = [vp, i64]
    L.lbcg_step.restype = C.c_int
    L.lbcg_moments.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, C.POINTER(C.c_double)]
    L.lbcg_moments.restype = C.c_int
    L.lbcg_free.argtypes = [vp]
    L.lbcg_free.restype = C.c_int
    L.lbcg_last_error.restype = C.c_char_p
    L.lbcg_steps_done.argtypes = [vp]
    L.lbcg_steps_done.restype = i64
    L.lbcg_index_map.argtypes = [vp, i32, vp, vp]
    L.lbcg_index_map.restype = C.c_int
    L.lbcg_get_populations.argtypes = [vp, i32, vp]
    L.lbcg_get_populations.restype = C.c_int
    L.lbcg_case_nodes.argtypes = [vp, i32]
    L.lbcg_case_nodes.restype = i64
    L.lbcg_storage_bytes.argtypes = [vp]
    L.lbcg_storage_bytes.restype = i32
    for name in ("lbcg_step_kernel", "lbcg_level_format", "lbcg_zchunk"):
        getattr(L, name).argtypes = [vp]
        getattr(L, name).restype = i32
    L.lbcg_timing.argtypes = [vp, i32]
    L.lbcg_timing.restype = C.c_int
    L.lbcg_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.lbcg_timing_read.restype = C.c_int
    L.lbcg_set_fields.argtypes = [vp, i32, C.POINTER(lbcg_fields)]
    L.lbcg_set_fields.restype = C.c_int
    L.lbcg_checkpoint_bytes.argtypes = [vp]
    L.lbcg_checkpoint_bytes.restype = i64
    L.lbcg_checkpoint_save.argtypes = [vp, vp, i64]
    L.lbcg_checkpoint_save.restype = C.c_int
    L.lbcg_checkpoint_load.argtypes = [vp, vp, i64]
    L.lbcg_checkpoint_load.restype = C.c_int
    _lib = L
    return L


def _check(rc):
    if rc != LBCG_OK:
        raise LbcgError(rc, load().lbcg_last_error().decode())
    return rc


def pack_case(p: dict) -> lbcg_case:
    c = lbcg_case()
    c.nx, c.ny, c.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    c.bc[:] = [int(v) for v in p["bc"]]
    for name in ("theta_deg", "rho_in", "alpha", "tau_v", "A", "force", "grav"):
        getattr(c, name)[:] = [float(v) for v in p[name]]
    for name in ("beta", "delta", "tau_e", "tau_q", "tau_pi", "rho_ref"):
        setattr(c, name, float(p[name]))
    c.improved = int(p["improved"])
    c.meq4 = int(p.get("meq4", 0))
    wu = p.get("wall_u", ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)))
    for side in range(2):
        c.wall_u[side][:] = [float(v) for v in wu[side]]
    return c


def _stream_ptr(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def lbcg_init(cases, storage="fp32", diag_every=0, block_nodes=0, persistent_blocks=0, kernel="auto",
              zchunk=0, graph_steps=0, level="auto", stream=None):
    """cases: list of (params, fields) from the workload generators; fields are
    host numpy arrays (FP64).  Returns the opaque handle (an int)."""
    L = load()
    n = len(cases)
    carr = (lbcg_case * n)(*[pack_case(p) for p, _ in cases])
    farr = (lbcg_fields * n)()
    keep = []
    for i, (p, fl) in enumerate(cases):
        N = int(p["nx"]) * int(p["ny"]) * int(p["nz"])
        ptrs = []
        for name in ("rhoR", "rhoB", "ux", "uy", "uz"):
            a = np.ascontiguousarray(fl[name], dtype=np.float64).reshape(-1)
            if a.size != N:
                raise ValueError(f"case {i}: field {name} has {a.size} values, expected {N}")
            keep.append(a)
            ptrs.append(a.ctypes.data)
        farr[i].rhoR, farr[i].rhoB, farr[i].ux, farr[i].uy, farr[i].uz = ptrs
        farr[i].on_device = 0
    opt = lbcg_options(STORAGE[storage] if isinstance(storage, str) else int(storage),
                       int(diag_every), int(block_nodes), int(persistent_blocks),
                       KERNEL[kernel] if isinstance(kernel, str) else int(kernel), int(zchunk),
                       int(graph_steps), LEVEL[level] if isinstance(level, str) else int(level))
    h = C.c_void_p()
    _check(L.lbcg_init(carr, n, farr, C.byref(opt), C.c_void_p(_stream_ptr(stream)), C.byref(h)))
    return h.value


def lbcg_step(h, nsteps):
    return _check(load().lbcg_step(C.c_void_p(h), int(nsteps)))


def lbcg_moments(h, case_id, rhoR=None, rhoB=None, rhoN=None, ux=None, uy=None, uz=None, diag=True):
    """Field arguments are torch CUDA float32 tensors (or None).  Returns the
    5 FP64 sums when diag is True (this synchronises the stream)."""
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    d = (C.c_double * 5)() if diag else None
    _check(load().lbcg_moments(C.c_void_p(h), int(case_id), ptr(rhoR), ptr(rhoB), ptr(rhoN), ptr(ux),
                               ptr(uy), ptr(uz), d))
    return np.array(list(d)) if diag else None


def lbcg_free(h):
    return _check(load().lbcg_free(C.c_void_p(h)))


def lbcg_last_error():
    return load().lbcg_last_error().decode()


def lbcg_steps_done(h):
    return int(load().lbcg_steps_done(C.c_void_p(h)))


def lbcg_case_nodes(h, case_id):
    return int(load().lbcg_case_nodes(C.c_void_p(h), int(case_id)))


def lbcg_storage_bytes(h):
    return int(load().lbcg_storage_bytes(C.c_void_p(h)))


def lbcg_step_kernel(h):
    """'fused' or 'twopass': the step kernel the handle resolved at init."""
    return {LBCG_KERNEL_FUSED: "fused", LBCG_KERNEL_TWOPASS: "twopass"}[int(load().lbcg_step_kernel(C.c_void_p(h)))]


def lbcg_level_format(h):
    """'pair' or 'compact': the level format the handle resolved at init."""
    return {LBCG_LEVEL_PAIR: "pair", LBCG_LEVEL_COMPACT: "compact"}[int(load().lbcg_level_format(C.c_void_p(h)))]


def lbcg_zchunk(h):
    """z-planes per fused tile the handle resolved at init (0: two-pass step)."""
    return int(load().lbcg_zchunk(C.c_void_p(h)))


def lbcg_set_fields(h, case_id, rhoR, rhoB, ux, uy, uz):
    """Reset a case to equilibrium from device (torch CUDA float64) fields."""
    f = lbcg_fields()
    keep = [t.contiguous() for t in (rhoR, rhoB, ux, uy, uz)]
    N = lbcg_case_nodes(h, case_id)
    for t in keep:
        if t.numel() != N or str(t.dtype) != "torch.float64" or not t.is_cuda:
            raise ValueError("fields must be CUDA float64 tensors of the case's node count")
    f.rhoR, f.rhoB, f.ux, f.uy, f.uz = [t.data_ptr() for t in keep]
    f.on_device = 1
    return _check(load().lbcg_set_fields(C.c_void_p(h), int(case_id), C.byref(f)))


def lbcg_timing(h, enable):
    return _check(load().lbcg_timing(C.c_void_p(h), int(bool(enable))))


def lbcg_timing_read(h):
    """{'aux'|'ghost'|'collide'|'fused': (total_ms, launches)} since the last read."""
    ms = (C.c_double * 4)()
    n = (C.c_int64 * 4)()
    _check(load().lbcg_timing_read(C.c_void_p(h), ms, n))
    return {k: (ms[i], int(n[i])) for i, k in enumerate(("aux", "ghost", "collide", "fused"))}


def lbcg_index_map(h, case_id):
    import torch
    N = lbcg_case_nodes(h, case_id)
    sn = torch.empty(19 * N, dtype=torch.int64, device="cuda")
    sd = torch.empty(19 * N, dtype=torch.int8, device="cuda")
    _check(load().lbcg_index_map(C.c_void_p(h), int(case_id), C.c_void_p(sn.data_ptr()),
                                 C.c_void_p(sd.data_ptr())))
    return sn.view(19, N), sd.view(19, N)


def lbcg_get_populations(h, case_id):
    import torch
    N = lbcg_case_nodes(h, case_id)
    f = torch.empty(2 * 19 * N, dtype=torch.float32, device="cuda")
    _check(load().lbcg_get_populations(C.c_void_p(h), int(case_id), C.c_void_p(f.data_ptr())))
    return f.view(2, 19, N)


def lbcg_checkpoint_save(h):
    """The handle's state image as a bytes object (host memory)."""
    n = int(load().lbcg_checkpoint_bytes(C.c_void_p(h)))
    if n < 0:
        raise LbcgError(LBCG_ESTATE, "invalid handle")
    buf = C.create_string_buffer(n)
    _check(load().lbcg_checkpoint_save(C.c_void_p(h), buf, n))
    return buf.raw


def lbcg_checkpoint_load(h, image: bytes):
    buf = C.create_string_buffer(image, len(image))
    return _check(load().lbcg_checkpoint_load(C.c_void_p(h), buf, len(image)))


class Solver:
    """Convenience owner of one handle: fields come back as torch tensors."""

    def __init__(self, cases, storage="fp32", **kw):
        self.cases = cases
        self.h = lbcg_init(cases, storage=storage, **kw)

    def step(self, n):
        lbcg_step(self.h, n)

    def fields(self, case_id=0):
        import torch
        N = lbcg_case_nodes(self.h, case_id)
        out = {k: torch.empty(N, dtype=torch.float32, device="cuda")
               for k in ("rhoR", "rhoB", "rhoN", "ux", "uy", "uz")}
        out["diag"] = lbcg_moments(self.h, case_id, out["rhoR"], out["rhoB"], out["rhoN"], out["ux"],
                                   out["uy"], out["uz"], diag=True)
        return out

    @property
    def steps(self):
        return lbcg_steps_done(self.h)

    def close(self):
        if self.h is not None:
            lbcg_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
