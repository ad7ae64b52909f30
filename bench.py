#!/usr/bin/env python
"""Throughput of the improved 3D colour-gradient LB step on one MI355X.

Workload: the Galilean droplet, a 128^3 periodic D3Q19 lattice, density and
viscosity ratio 1, droplet radius 20 at a seeded random centre, uniform
initial velocity (0.05, 0.05, 0.05), tau_v drawn in [0.6, 1.0] from the seed,
plain FP32 populations.  A step is one full time step of the method (moments,
colour gradient, MRT collision with correction term and perturbation,
recoloring, streaming).  Prints one JSON line.

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
# Algorithmic HBM bytes per node of one launch of the collision pass: read 38
# population deviations and the writers' stored (rho_R, rho_B) (8 B per node),
# read the node's aux value (rho^N, Qbar: 16 B), write 38 deviations and the
# node's (rho_R, rho_B).
POP = {"fp32": 4, "fp16s": 2, "bf16s": 2}
COLLIDE_BYTES = {k: 38 * b + 8 + 16 + 38 * b + 8 for k, b in POP.items()}
# The fused single-pass step: populations and stored densities read and
# written once (the phase-field halo lives in LDS).
FUSED_BYTES = {k: 2 * (38 * b + 8) for k, b in POP.items()}
# The method's own minimum per node and step in this storage: populations and
# stored densities read and written once.
STEP_BYTES = {k: 2 * (38 * b + 8) for k, b in POP.items()}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "d3q19.hpp"):
        with open(os.path.join(ROOT, "paper_1904_03618_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage, kernel):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, only if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{storage}_galilean128_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def dominant(kt, storage):
    """(name, avg ms, algorithmic bytes per node) of the kernel that dominates a step."""
    if kt["fused"][1]:
        return "k_fused", kt["fused"][0] / kt["fused"][1], FUSED_BYTES[storage]
    return "k_collide", kt["collide"][0] / kt["collide"][1], COLLIDE_BYTES[storage]


def run_form(B, cases, storage, steps, warmup, timing=True, kernel="auto", kernel_steps=200, repeats=0,
             repeat_steps=200):
    """Time `steps` steps (no per-kernel events inside the timed region), then,
    if timing, `kernel_steps` more steps with HIP event pairs around every
    kernel for the per-kernel averages.  Fields are taken after the timed
    steps.  With repeats > 0, also time that many further runs of
    repeat_steps steps each (ms per step of each run, returned as kt["repeats"])."""
    import torch
    s = B.Solver(cases, storage=storage, kernel=kernel)
    try:
        s.step(warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        fl = {k: v.double() for k, v in s.fields(0).items() if k != "diag"}
        reps = []
        for _ in range(repeats):
            e0.record()
            s.step(repeat_steps)
            e1.record()
            torch.cuda.synchronize()
            reps.append(e0.elapsed_time(e1) / repeat_steps)
        kt = None
        if timing:
            B.lbcg_timing(s.h, 1)
            B.lbcg_timing_read(s.h)
            s.step(kernel_steps)
            kt = B.lbcg_timing_read(s.h)
            kt["repeats"] = reps
        return ms, kt, fl
    finally:
        s.close()


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
    picked by the autotuner.  Aggregate MLUPS over all boxes."""
    import torch
    from paper_1904_03618_amd import autotune as AT
    from paper_1904_03618_amd import workloads as W
    t0 = time.time()
    cases = W.impact_batch(ncases)
    gen_s = time.time() - t0
    N = sum(p["nx"] * p["ny"] * p["nz"] for p, _ in cases)
    opts, rep = AT.autotune(cases, storage)
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
    return {"workload": f"{ncases} droplet-impact boxes, sides 48..128 (seeded), wetting bottom wall",
            "storage": storage, "nodes": N, "MLUPS": N / ms / 1e3, "ms_per_step": ms, "steps": steps,
            "warmup": warmup, "options": opts, "autotune_key": rep["key"], "autotune_cached": rep["cached"],
            "cases_non_finite": bad, "input_generation_s": gen_s}


def cpu_baseline(p, fl, budget_s):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload (the full 128^3 lattice for a few steps)."""
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
    out = {"value": N * n / dt / 1e6, "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
           "sample": f"galilean droplet 128^3, FP64 oracle, {n} timed steps after 1 untimed "
                     f"({dt:.1f} s)"}
    out["one_core"] = cpu_one_core()
    return out


def cpu_one_core():
    """The same oracle on one core (one step of the full lattice), in a child
    process started with OMP_NUM_THREADS=1 (the thread count is fixed when
    OpenMP starts); the child never touches the GPU."""
    import subprocess
    code = ("import json, sys, time\n"
            f"sys.path.insert(0, {ROOT!r})\n"
            "from oracle import oracle as O\n"
            "from paper_1904_03618_amd import workloads as W\n"
            "p, fl = W.galilean_droplet(128, 20.0, seed=1904)\n"
            "f = O.init(p, fl['rhoR'], fl['rhoB'], fl['ux'], fl['uy'], fl['uz'])\n"
            "t = time.time(); O.run(p, f, 1); dt = time.time() - t\n"
            "print(json.dumps({'value': 128 ** 3 / dt / 1e6, 'unit': 'MLUPS', 'cores': O.threads(),\n"
            "                  'sample': f'one step of the full lattice ({dt:.1f} s)'}))\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        return json.loads(r.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        return {"error": str(e)[:200]}


MFMA_BF16_PEAK_TFLOPS = 2500.0


def surrogate_bench(with_rt):
    """The learned surrogate (BF16 MFMA U-Net): full-domain inference on the
    128 x 128 x 512 Rayleigh-Taylor box and a training step on four 64^3
    crops, against the dense BF16 matrix-core peak; optionally the gated
    hybrid on a 32 x 32 x 128 Rayleigh-Taylor run (train, then jump 100 steps
    at a time while the bubble and spike fronts stay within 1 lattice unit of
    the LB run) with its time-to-solution gain over plain LB."""
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
        rt = R.experiment(L=32, gates=(1.0,))
        g = rt["gates"]["1.0"]
        res["rt_hybrid"] = {
            "lattice": rt["lattice"], "jump_steps": rt["every"], "heal_steps": rt["heal"], "steps": rt["steps"],
            "train_amps": rt["train_amps"], "val_amp": rt["val_amp"], "eval_amp": rt["eval_amp"],
            "train_iters": rt["train_iters"], "seeds": rt["seeds"], "selected_seed": rt["selected_seed"],
            "selected_after": rt["selected_after"], "validation": rt["validation"],
            "train_s": rt["train_s"], "loss_first": rt["loss_first"],
            "loss_last": rt["loss_last"], "gate_lu": 1.0, "accepted": g["accepted"], "jumps": g["jumps"],
            "max_accepted_front_error": g["max_accepted_error"], "final_front_error": g["final_front_error"],
            "lb_s": rt["lb_s"], "hybrid_s": g["hybrid_s"], "gain": g["gain"],
            "persistence": g["persistence"]}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--forms", default="fp16s,bf16s", help="extra storage forms to time ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", default="auto", choices=["auto", "twopass", "fused"])
    ap.add_argument("--batch-steps", type=int, default=100, help="timed steps of the impact batch (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--surrogate", type=int, default=1, help="time the surrogate network (1) or skip it (0)")
    ap.add_argument("--surrogate-rt", type=int, default=1,
                    help="run the gated surrogate/LB hybrid on a 32x32x128 Rayleigh-Taylor case (0: skip)")
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
    p, fl = W.galilean_droplet(128, 20.0, seed=1904)
    N = p["nx"] * p["ny"] * p["nz"]
    cases = [(p, fl)]

    ms, kt, ref = run_form(B, cases, "fp32", args.steps, args.warmup, kernel=args.kernel, repeats=5)
    reps = kt.pop("repeats")
    ms_step = ms / args.steps
    mlups = N * args.steps / (ms * 1e-3) / 1e6
    kname, avg_col, kbytes = dominant(kt, "fp32")
    ach = kbytes * N / (avg_col * 1e-3) / 1e9
    traffic = measured_traffic("fp32", kname)

    forms = {}
    for st in [s for s in args.forms.split(",") if s]:
        fms, fkt, ff = run_form(B, cases, st, args.steps, args.warmup, kernel=args.kernel)
        fname, f_avg, f_bytes = dominant(fkt, st)
        err_n = float((ff["rhoN"] - ref["rhoN"]).abs().max())
        err_u = float(max((ff[k] - ref[k]).abs().max() for k in ("ux", "uy", "uz")))
        forms[st] = {"MLUPS": N * args.steps / (fms * 1e-3) / 1e6, "ms_per_step": fms / args.steps,
                     "kernel": fname, "kernel_avg_ms": f_avg,
                     "kernel_GBps": f_bytes * N / (f_avg * 1e-3) / 1e9,
                     "max_abs_diff_vs_fp32_after_steps": {"rhoN": err_n, "u": err_u,
                                                          "steps": args.steps + args.warmup}}

    copy = copy_probe(args.copy_probe_mib) if args.copy_probe_mib > 0 else None
    sur = surrogate_bench(args.surrogate_rt) if args.surrogate else None
    batch = batch_bench(B, args.batch_steps, 10) if args.batch_steps > 0 else None

    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "galilean droplet 128^3 (periodic, R=20, u0=0.05, seed 1904)",
                   "lattice": [128, 128, 128], "storage": "fp32", "tau_v": p["tau_v"][0],
                   "parallelism": "single GPU"},
        "step_algorithmic_GBps": mlups * 1e6 * STEP_BYTES["fp32"] / 1e9,
        "repeat_runs": {"runs": len(reps), "steps": 200, "ms_per_step": reps,
                        "median_MLUPS": N / (float(np.median(reps)) * 1e-3) / 1e6},
        "kernels_avg_ms": {k: v[0] / v[1] for k, v in kt.items() if v[1]},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBPS, "kernel": kname + "<fp32>",
                     "bytes_per_node": kbytes, "traffic": traffic},
        "forms": forms,
    }
    if batch:
        out["batch"] = batch
    if sur:
        out["surrogate"] = sur
    if copy:
        out["copy_probe"] = copy
        out["roofline"]["frac_of_copy_probe"] = ach / copy["GBps"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, fl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
