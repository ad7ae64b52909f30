"""Launch-shape autotuner for the batched step.

For a list of cases and a storage format it times each candidate launch
configuration (step kernel, workgroup tile, persistent grid, z-chunk, graph
capture) on a scratch handle built from a sample of the cases, and returns the
fastest as keyword options for ``lbcg_init``.  Results are cached in a JSON
file in the user's cache directory (``LBCG_AUTOTUNE_CACHE`` overrides it),
keyed by the box-size class of the cases and the storage format, so a later
run on the same machine with the same kind of workload reuses the choice
without timing; ``cache=None`` times every call.
"""
from __future__ import annotations

import json
import os

DEFAULT_CACHE = os.environ.get("LBCG_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "lbcg", "autotune.json"))


def _moving(p):
    return any(v != 0.0 for side in p.get("wall_u", ()) for v in side)


def box_class(cases, storage):
    """Cache key: storage, number of cases, wall/periodic mix, the node count
    rounded to two significant digits, and the number of cases with moving
    walls when there are any (those run another instantiation of the step
    kernels)."""
    n = sum(int(p["nx"]) * int(p["ny"]) * int(p["nz"]) for p, _ in cases)
    walls = sum(1 for p, _ in cases if any(p["bc"]))
    lo = min(min(p["nx"], p["ny"], p["nz"]) for p, _ in cases)
    hi = max(max(p["nx"], p["ny"], p["nz"]) for p, _ in cases)
    key = f"{storage}|cases={len(cases)}|walls={walls}|side={lo}-{hi}|nodes={float(f'{n:.2g}'):.3g}"
    moving = sum(1 for p, _ in cases if _moving(p))
    return key + (f"|moving={moving}" if moving else "")


def candidates(eligible_fused):
    """Launch shapes to time: the two-pass step (256- or 128-node tiles,
    with or without a persistent grid) and, where the cases allow it, the
    fused step at 16-, 32- and 64-plane chunks; each with and without an
    8-step graph."""
    out = []
    for block in (256, 128):
        for persistent in (0, 1024):
            for graph in (0, 8):
                out.append(dict(kernel="twopass", block_nodes=block, persistent_blocks=persistent,
                                graph_steps=graph))
    if eligible_fused:
        for zc in (16, 32, 64):
            for graph in (0, 8):
                out.append(dict(kernel="fused", zchunk=zc, persistent_blocks=0, graph_steps=graph))
    return out


def _fused_ok(cases):
    """The fused kernel takes boxes without walls or with walls on z (any
    contact angle, at rest or moving)."""
    return all(not (p["bc"][0] or p["bc"][1]) for p, _ in cases)


def time_config(B, cases, storage, opts, steps=24, warmup=8):
    import torch
    s = B.Solver(cases, storage=storage, **opts)
    try:
        s.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps
    finally:
        s.close()


def autotune(cases, storage="fp16s", sample_every=8, steps=24, warmup=8, cache=DEFAULT_CACHE,
             retune=False, log=None):
    """Return (options dict, report).  Times every candidate on every
    `sample_every`-th case (at least 8 cases) and caches the winner."""
    from . import lbcg as B
    key = box_class(cases, storage)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if key in table and not retune:
        return dict(table[key]["options"]), {"key": key, "cached": True}
    sample = cases[::sample_every] if len(cases) >= 8 * sample_every else cases
    nodes = sum(int(p["nx"]) * int(p["ny"]) * int(p["nz"]) for p, _ in sample)
    results = []
    for opts in candidates(_fused_ok(cases)):
        ms = time_config(B, sample, storage, opts, steps=steps, warmup=warmup)
        results.append({"options": opts, "ms_per_step": ms, "MLUPS": nodes / ms / 1e3})
        if log:
            log(f"autotune {opts} -> {ms:.4f} ms/step, {nodes / ms / 1e3:.0f} MLUPS")
    best = min(results, key=lambda r: r["ms_per_step"])
    table[key] = {"options": best["options"], "sample_nodes": nodes, "trials": results}
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1)
        os.replace(tmp, cache)
    return dict(best["options"]), {"key": key, "cached": False, "trials": results}
