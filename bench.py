#!/usr/bin/env python
"""Throughput of the improved 3D colour-gradient LB step on one MI355X.

Headline workload: the 3D Rayleigh-Taylor instability (Sec. IV.C) on a
128 x 128 x 512 D3Q19 lattice, walls on z, periodic sides, Atwood number 0.5
(rho^in 3/1), gravity 2e-5, Re = 1024, single-mode perturbation of amplitude
0.05 L, FP32 arithmetic and storage; the largest single-GPU configuration of the
benchmark set.  A step is one full time step of the method (moments, colour
gradient, MRT collision with correction term and perturbation, recoloring,
streaming with bounce-back walls).  Beside it: the same case scaled to
256 x 256 x 1024, the 16-bit storage forms, the 128^3 Galilean droplet, the
batch of 256 droplet-impact boxes (launch shape tuned on the spot), the
learned surrogate, a copy probe and the FP64 oracle on the host cores.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + HBM GB/s (% peak): FP32 plain vs FP16-store/surrogate at stated error"
HBM_PEAK_GBPS = 8000.0
POP = {"fp32": 4, "fp16s": 2, "bf16s": 2}
# Algorithmic HBM bytes per fluid node and step of the method: 38
# populations read and 38 written (the figure the roofline is priced at).
ALGO_BYTES = {k: 2 * 38 * b for k, b in POP.items()}
# What the fused step moves by design, per level format: pairs move the 38
# populations plus the colour densities each writer stores with them (8 B
# read, 8 B written); the compact format moves 20 population values (the
# rest pair and 18 totals) plus 7 FP32 words of writer data, read and written.
FUSED_BYTES = {"pair": {k: 2 * (38 * b + 8) for k, b in POP.items()},
               "compact": {k: 2 * (20 * b + 28) for k, b in POP.items()}}
# The two-pass step: populations and stored densities read twice (moments
# pass, collision pass), the aux value written once and read once.
TWOPASS_BYTES = {k: 3 * (38 * b + 8) + 2 * 16 for k, b in POP.items()}
KERNEL_INDEX = {"aux": "k_aux", "ghost": "k_ghost", "collide": "k_collide", "fused": "k_fused"}


def kernel_source_hash():
    """Hash of the step kernels' code (comments and blank lines left out, so
    that a comment edit does not invalidate a counter profile)."""
    import re
    h = hashlib.sha256()
    for f in ("kernels.hpp", "d3q19.hpp"):
        with open(os.path.join(ROOT, "paper_1904_03618_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel, storage, workload):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, only if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{storage}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return {"bytes_per_launch": d["bytes_per_launch"], "bytes_per_node": d["bytes_per_node"],
            "file": os.path.relpath(path, ROOT)}


def timed_run(B, cases, storage, steps, warmup, kernel_steps=100, repeats=0, repeat_steps=200, layout=None,
              **opts):
    """Time `steps` steps with HIP events on the handle's stream (no
    per-kernel events inside), then `repeats` further runs, then
    `kernel_steps` steps with event pairs around every kernel.  Returns
    (ms per step, per-kernel average ms, repeat ms list, fields of case 0
    after the timed steps); `layout` (a dict) receives the step kernel and
    level format the handle resolved."""
    import torch
    s = B.Solver(cases, storage=storage, **opts)
    if layout is not None:
        layout.update(kernel=B.lbcg_step_kernel(s.h), level=B.lbcg_level_format(s.h), zchunk=B.lbcg_zchunk(s.h))
    try:
        stream = torch.cuda.current_stream()
        s.step(warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        s.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        fl = {k: v.double() for k, v in s.fields(0).items() if k != "diag"}
        reps = []
        for _ in range(repeats):
            e0.record(stream)
            s.step(repeat_steps)
            e1.record(stream)
            torch.cuda.synchronize()
            reps.append(e0.elapsed_time(e1) / repeat_steps)
        kt = {}
        if kernel_steps and not opts.get("graph_steps"):
            B.lbcg_timing(s.h, 1)
            B.lbcg_timing_read(s.h)
            s.step(kernel_steps)
            raw = B.lbcg_timing_read(s.h)
            kt = {KERNEL_INDEX[k]: v[0] / v[1] for k, v in raw.items() if v[1]}
        return ms, kt, reps, fl
    finally:
        s.close()


def roofline(kernels, storage, N, ms_step, level="pair"):
    """Roofline of the dominant kernel (the fused step, or the two-pass
    collision pass) at the method's algorithmic bytes, and the step's."""
    if "k_fused" in kernels:
        name, kms, design = "k_fused", kernels["k_fused"], FUSED_BYTES[level][storage]
    else:
        name, kms, design = "k_collide", kernels.get("k_collide", ms_step), TWOPASS_BYTES[storage]
    ach = ALGO_BYTES[storage] * N / (kms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS,
            "kernel": f"{name}<{storage}>", "level_format": level if name == "k_fused" else "pair",
            "kernel_avg_ms": kms, "bytes_per_node": ALGO_BYTES[storage],
            "design_bytes_per_node": design if name == "k_fused" else None,
            "design_GBps": design * N / (kms * 1e-3) / 1e9 if name == "k_fused" else None,
            "step_achieved": ALGO_BYTES[storage] * N / (ms_step * 1e-3) / 1e9,
            "step_frac": ALGO_BYTES[storage] * N / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def copy_probe(mib):
    """Attainable HBM rate: a plain device-to-device copy of `mib` MiB (read +
    write counted), timed with HIP events."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 10
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return {"bytes": 2 * mib * (1 << 20), "avg_ms": ms, "GBps": 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9}


def batch_bench(B, steps, warmup, storage="fp16s", ncases=256):
    """Batched droplet impact: `ncases` independent boxes of side 48..128 in one
    handle (one launch per kernel over every box), FP16S storage, launch shape
    picked by the autotuner on this machine (timed now, not read from a cache).
    Aggregate MLUPS over all boxes and the step's roofline."""
    import torch
    from paper_1904_03618_amd import autotune as AT
    from paper_1904_03618_amd import workloads as W
    t0 = time.time()
    cases = W.impact_batch(ncases)
    gen_s = time.time() - t0
    N = sum(p["nx"] * p["ny"] * p["nz"] for p, _ in cases)
    t0 = time.time()
    opts, rep = AT.autotune(cases, storage, cache=None, retune=True)
    tune_s = time.time() - t0
    s = B.Solver(cases, storage=storage, diag_every=0, **opts)
    try:
        s.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        bad = sum(1 for c in range(ncases) if not np.isfinite(B.lbcg_moments(s.h, c)).all())
    finally:
        s.close()
    ach = ALGO_BYTES[storage] * N / (ms * 1e-3) / 1e9
    trials = [{"options": t["options"], "MLUPS_sample": t["MLUPS"]} for t in rep.get("trials", [])]
    return {"workload": f"{ncases} droplet-impact boxes, sides 48..128 (seeded), wetting bottom wall",
            "storage": storage, "nodes": N, "MLUPS": N / ms / 1e3, "ms_per_step": ms, "steps": steps,
            "warmup": warmup, "options": opts, "autotune": {"key": rep["key"], "cached": rep["cached"],
                                                             "tuned_here_s": tune_s, "trials": trials},
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBPS, "level": "step", "bytes_per_node": ALGO_BYTES[storage]},
            "cases_non_finite": bad, "input_generation_s": gen_s}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(p, fl, budget_s, label):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: the full lattice for as many steps as fit the budget."""
    from oracle import oracle as O
    f = O.init(p, fl["rhoR"], fl["rhoB"], fl["ux"], fl["uy"], fl["uz"])
    N = p["nx"] * p["ny"] * p["nz"]
    t = time.time()
    O.run(p, f, 1)
    dt1 = time.time() - t
    n = max(1, min(50, int(budget_s / max(dt1, 1e-3)) - 1))
    t = time.time()
    O.run(p, f, n)
    dt = time.time() - t
    del f
    return {"value": N * n / dt / 1e6, "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "sample": f"{label}, FP64 oracle, {n} timed steps of the full lattice after 1 untimed ({dt:.1f} s)"}


MFMA_BF16_PEAK_TFLOPS = 2500.0


def surrogate_bench(with_rt):
    """The learned surrogate (BF16 MFMA U-Net): full-domain inference on the
    128 x 128 x 512 Rayleigh-Taylor box and a training step on four 64^3
    crops, against the dense BF16 matrix-core peak; optionally the gated
    hybrid on a Rayleigh-Taylor run with its time-to-solution against plain LB."""
    from paper_1904_03618_amd import surrogate as S
    inf = S.bench_unet((1, 512, 128, 128), iters=5, train=False)
    tr = S.bench_unet((4, 64, 64, 64), iters=5, train=True)
    res = {
        "inference": {"shape": inf["shape"], "ms": inf["forward_ms"], "gflop": inf["forward_gflop"],
                      "roofline": {"bound": "mfma", "achieved": inf["forward_tflops"], "peak": MFMA_BF16_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": inf["forward_tflops"] / MFMA_BF16_PEAK_TFLOPS}},
        "training_step": {"shape": tr["shape"], "ms": tr["train_ms"], "gflop": tr["train_gflop"],
                          "TFLOPs": tr["train_tflops"]},
        "params": inf["params"],
    }
    if with_rt:
        from paper_1904_03618_amd import surrogate_rt as R
        res["rt_hybrid"] = R.bench_summary(R.experiment(L=32, gates=(1.0,)))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--forms", default="fp16s,bf16s", help="extra storage forms to time ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", default="auto", choices=["auto", "twopass", "fused"])
    ap.add_argument("--large", type=int, default=1, help="also time the 256 x 256 x 1024 box (0: skip)")
    ap.add_argument("--galilean", type=int, default=1, help="also time the 128^3 Galilean droplet (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=100, help="timed steps of the impact batch (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--repeats", type=int, default=5, help="further 200-step runs of the headline case")
    ap.add_argument("--surrogate", type=int, default=1, help="time the surrogate network (1) or skip it (0)")
    ap.add_argument("--surrogate-rt", type=int, default=1,
                    help="run the gated surrogate/LB hybrid on a Rayleigh-Taylor case (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=1024,
                    help="size of the device copy that measures the attainable HBM rate (0: skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the step runs on a single MI355X; "
              "multi-GPU slab decomposition is not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_03618_amd import lbcg as B
    from paper_1904_03618_amd import workloads as W

    torch.cuda.set_device(0)
    label = "rayleigh-taylor 128x128x512"
    p, fl = W.rayleigh_taylor(128)
    N = p["nx"] * p["ny"] * p["nz"]
    cases = [(p, fl)]

    lay = {}
    ms, kt, reps, ref = timed_run(B, cases, "fp32", args.steps, args.warmup, repeats=args.repeats, layout=lay,
                                  kernel=args.kernel)
    mlups = N / (ms * 1e-3) / 1e6
    roof = roofline(kt, "fp32", N, ms, lay["level"])
    roof["traffic"] = measured_traffic(roof["kernel"].split("<")[0], "fp32", "rt128x128x512")

    forms = {}
    for st in [s for s in args.forms.split(",") if s]:
        flay = {}
        fms, fkt, _, ff = timed_run(B, cases, st, args.steps, args.warmup, layout=flay, kernel=args.kernel)
        err_n = float((ff["rhoN"] - ref["rhoN"]).abs().max())
        err_u = float(max((ff[k] - ref[k]).abs().max() for k in ("ux", "uy", "uz")))
        froof = roofline(fkt, st, N, fms, flay["level"])
        froof["traffic"] = measured_traffic(froof["kernel"].split("<")[0], st, "rt128x128x512")
        forms[st] = {"MLUPS": N / (fms * 1e-3) / 1e6, "ms_per_step": fms, "zchunk": flay["zchunk"],
                     "kernels_avg_ms": fkt,
                     "roofline": froof, "vs_fp32": N / (fms * 1e-3) / 1e6 / mlups,
                     "max_abs_diff_vs_fp32_after_steps": {"rhoN": err_n, "u": err_u,
                                                          "steps": args.steps + args.warmup}}

    extra = {}
    if args.large:
        pl, fll = W.rayleigh_taylor(256)
        NL = pl["nx"] * pl["ny"] * pl["nz"]
        big = {}
        for st in ("fp32", "fp16s"):
            llay = {}
            lms, lkt, _, _ = timed_run(B, [(pl, fll)], st, min(args.steps, 100), 5, kernel_steps=20, layout=llay,
                                       kernel=args.kernel)
            big[st] = {"MLUPS": NL / (lms * 1e-3) / 1e6, "ms_per_step": lms, "zchunk": llay["zchunk"],
                       "kernels_avg_ms": lkt,
                       "roofline": roofline(lkt, st, NL, lms, llay["level"])}
        del fll
        extra["rayleigh_taylor_256x256x1024"] = big
    if args.galilean:
        pg, flg = W.galilean_droplet(128, 20.0, seed=1904)
        NG = 128 ** 3
        gal = {}
        for st in ("fp32", "fp16s"):
            glay = {}
            gms, gkt, _, _ = timed_run(B, [(pg, flg)], st, args.steps, args.warmup, layout=glay, kernel=args.kernel)
            gal[st] = {"MLUPS": NG / (gms * 1e-3) / 1e6, "ms_per_step": gms, "zchunk": glay["zchunk"],
                       "kernels_avg_ms": gkt,
                       "roofline": roofline(gkt, st, NG, gms, glay["level"])}
        extra["galilean_droplet_128"] = gal

    copy = copy_probe(args.copy_probe_mib) if args.copy_probe_mib > 0 else None
    sur = surrogate_bench(args.surrogate_rt) if args.surrogate else None
    batch = batch_bench(B, args.batch_steps, 10) if args.batch_steps > 0 else None

    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rayleigh-taylor 128x128x512 (walls on z, At 0.5, g 2e-5, Re 1024, amplitude 0.05 L)",
                   "lattice": [128, 128, 512], "storage": "fp32", "kernel": lay["kernel"],
                   "level_format": lay["level"], "zchunk": lay["zchunk"],
                   "tau_v": list(p["tau_v"]), "parallelism": "single GPU"},
        "repeat_runs": {"runs": len(reps), "steps": 200, "ms_per_step": reps,
                        "median_MLUPS": N / (float(np.median(reps)) * 1e-3) / 1e6 if reps else None},
        "kernels_avg_ms": kt,
        "roofline": roof,
        "forms": forms,
    }
    out.update(extra)
    if batch:
        out["batch"] = batch
    if sur:
        out["surrogate"] = sur
    if copy:
        out["copy_probe"] = copy
        out["roofline"]["frac_of_copy_probe_design_bytes"] = (roof["design_GBps"] / copy["GBps"]
                                                              if roof.get("design_GBps") else None)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, fl, args.cpu_seconds, label)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
