"""ctypes wrapper of the FP64 CPU oracle (``lbcg_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module; the product path never imports it.

Parameters are the plain dict produced by the seeded workload generators (keys
listed in ``PARAM_KEYS``); fields are numpy arrays in x-fastest node order.
Populations use the layout f[k, i, node] (k = 0 red, 1 blue; i = 0..18 as in
Eq. (5) of the paper).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbcg_oracle.c")
LIB = os.path.join(HERE, "liblbcg_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("bc", C.c_int * 3),
        ("theta_deg", C.c_double * 2),
        ("rho_in", C.c_double * 2),
        ("alpha", C.c_double * 2),
        ("tau_v", C.c_double * 2),
        ("A", C.c_double * 2),
        ("beta", C.c_double), ("delta", C.c_double),
        ("tau_e", C.c_double), ("tau_q", C.c_double), ("tau_pi", C.c_double),
        ("force", C.c_double * 3), ("grav", C.c_double * 3), ("rho_ref", C.c_double),
        ("improved", C.c_int),
        ("meq4", C.c_int),
        ("wall_u", (C.c_double * 3) * 2),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(_Params)
        L.orc_tables.argtypes = [dp, dp, dp, C.POINTER(C.c_int), dp, dp]
        L.orc_feq.argtypes = [pp, C.c_int, C.c_double, dp, dp]
        L.orc_tau_v.argtypes = [pp, C.c_double]
        L.orc_tau_v.restype = C.c_double
        L.orc_collide_color.argtypes = [pp, C.c_int, dp, C.c_double, C.c_double, dp,
                                        C.c_double, dp, dp, dp, dp]
        L.orc_recolor.argtypes = [pp, dp, C.c_double, C.c_double, dp, dp, dp]
        L.orc_init.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.orc_run.argtypes = [pp, dp, C.c_int64]
        L.orc_run.restype = C.c_int
        L.orc_fields.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_fields.restype = C.c_int
        L.orc_index_map.argtypes = [pp, C.POINTER(C.c_int64), C.POINTER(C.c_int8)]
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


PARAM_DEFAULTS = dict(bc=(0, 0, 0), theta_deg=(90.0, 90.0), beta=0.5, delta=0.98,
                      tau_e=1.0, tau_q=1.0, tau_pi=1.0, force=(0.0, 0.0, 0.0),
                      grav=(0.0, 0.0, 0.0), rho_ref=0.0, improved=1, meq4=0,
                      wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)))


def make_params(p: dict) -> _Params:
    q = dict(PARAM_DEFAULTS)
    q.update(p)
    s = _Params()
    s.nx, s.ny, s.nz = int(q["nx"]), int(q["ny"]), int(q["nz"])
    for name in ("bc",):
        getattr(s, name)[:] = [int(v) for v in q[name]]
    for name in ("theta_deg", "rho_in", "alpha", "tau_v", "A", "force", "grav"):
        getattr(s, name)[:] = [float(v) for v in q[name]]
    for name in ("beta", "delta", "tau_e", "tau_q", "tau_pi", "rho_ref"):
        setattr(s, name, float(q[name]))
    s.improved = int(q["improved"])
    s.meq4 = int(q["meq4"])
    for side in range(2):
        s.wall_u[side][:] = [float(v) for v in q["wall_u"][side]]
    return s


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def tables():
    """(e[19,3], w[19], B[19], opp[19], M[19,19], Minv[19,19]) as the oracle builds them."""
    e = np.zeros((19, 3)); w = np.zeros(19); b = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32); M = np.zeros((19, 19)); Mi = np.zeros((19, 19))
    lib().orc_tables(_dp(e), _dp(w), _dp(b), opp.ctypes.data_as(C.POINTER(C.c_int)), _dp(M), _dp(Mi))
    return e, w, b, opp, M, Mi


def feq(params: dict, k: int, rho: float, u) -> np.ndarray:
    out = np.zeros(19)
    s = make_params(params)
    lib().orc_feq(C.byref(s), k, rho, _dp(_f64(u)), _dp(out))
    return out


def tau_v(params: dict, rhoN: float) -> float:
    s = make_params(params)
    return lib().orc_tau_v(C.byref(s), float(rhoN))


def collide_color(params, k, f, rho_k, rho, u, tau, grad, Qk, F):
    s = make_params(params)
    out = np.zeros(19)
    lib().orc_collide_color(C.byref(s), k, _dp(_f64(f)), rho_k, rho, _dp(_f64(u)), tau,
                            _dp(_f64(grad)), _dp(_f64(Qk)), _dp(_f64(F)), _dp(out))
    return out


def recolor(params, fstar, rhoR, rhoB, grad):
    s = make_params(params)
    oR = np.zeros(19); oB = np.zeros(19)
    lib().orc_recolor(C.byref(s), _dp(_f64(fstar)), rhoR, rhoB, _dp(_f64(grad)), _dp(oR), _dp(oB))
    return oR, oB


def init(params: dict, rhoR0, rhoB0, ux0, uy0, uz0) -> np.ndarray:
    """Equilibrium start f^k = f^{k,eq}(rho_k, u0); returns f[2, 19, N]."""
    s = make_params(params)
    N = s.nx * s.ny * s.nz
    f = np.zeros((2, 19, N))
    arrs = [_f64(a).reshape(-1) for a in (rhoR0, rhoB0, ux0, uy0, uz0)]
    for a in arrs:
        assert a.size == N
    lib().orc_init(C.byref(s), *[_dp(a) for a in arrs], _dp(f))
    return f


def run(params: dict, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance f in place by nsteps; returns f."""
    assert f.dtype == np.float64 and f.flags.c_contiguous
    s = make_params(params)
    assert f.size == 2 * 19 * s.nx * s.ny * s.nz
    if lib().orc_run(C.byref(s), _dp(f), int(nsteps)) != 0:
        raise MemoryError("oracle allocation failed")
    return f


def fields(params: dict, f: np.ndarray) -> dict:
    """rhoR, rhoB, ux, uy, uz, rhoN, grad[N,3], Q[N,2,3], diag[5] of the current level."""
    s = make_params(params)
    N = s.nx * s.ny * s.nz
    out = {k: np.zeros(N) for k in ("rhoR", "rhoB", "ux", "uy", "uz", "rhoN")}
    grad = np.zeros((N, 3)); Qk = np.zeros((N, 2, 3)); diag = np.zeros(5)
    rc = lib().orc_fields(C.byref(s), _dp(_f64(f)), *[_dp(out[k]) for k in
                          ("rhoR", "rhoB", "ux", "uy", "uz", "rhoN")], _dp(grad), _dp(Qk), _dp(diag))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    out.update(grad=grad, Q=Qk, diag=diag)
    return out


def index_map(params: dict):
    """(src_node[19, N] int64, src_dir[19, N] int8): the pull source of every (i, node)."""
    s = make_params(params)
    N = s.nx * s.ny * s.nz
    sn = np.zeros((19, N), dtype=np.int64); sd = np.zeros((19, N), dtype=np.int8)
    lib().orc_index_map(C.byref(s), sn.ctypes.data_as(C.POINTER(C.c_int64)),
                        sd.ctypes.data_as(C.POINTER(C.c_int8)))
    return sn, sd


def threads() -> int:
    return int(lib().orc_threads())
