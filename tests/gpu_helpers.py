"""Shared helpers of the GPU parity tests: run a list of cases through the C
ABI and the same cases through the FP64 oracle, and compare."""
import numpy as np

FIELDS = ("rhoR", "rhoB", "rhoN", "ux", "uy", "uz")


def gpu_run(cases, steps, storage="fp32", **opt):
    """Run cases (list of (params, fields)) for `steps` steps on the GPU in one
    handle; returns a list of dicts of numpy float64 arrays + 'diag'."""
    import torch
    from paper_1904_03618_amd import lbcg as B
    s = B.Solver(cases, storage=storage, **opt)
    try:
        if steps:
            s.step(steps)
        out = []
        for c in range(len(cases)):
            fl = s.fields(c)
            torch.cuda.synchronize()
            out.append({k: (v.double().cpu().numpy() if k != "diag" else v) for k, v in fl.items()})
        return out
    finally:
        s.close()


def oracle_run(p, fl, steps):
    from oracle import oracle as O
    f = O.init(p, fl["rhoR"], fl["rhoB"], fl["ux"], fl["uy"], fl["uz"])
    if steps:
        O.run(p, f, steps)
    return O.fields(p, f)


def max_err(g, o):
    return {k: float(np.abs(g[k] - o[k]).max()) for k in FIELDS}


def report(tag, e):
    print(tag, " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
