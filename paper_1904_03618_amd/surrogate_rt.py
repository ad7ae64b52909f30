"""The learned surrogate on the Rayleigh-Taylor runs (Sec. IV.C workload).

Pipeline
  1. snapshots: the LB solver (include/lbcg.h) runs Rayleigh-Taylor cases and
     records (rho^N, u) every `every` steps;
  2. training: the U-Net (surrogate.py) learns the map from the fields at t
     to the fields at t + every on the snapshots (whole box, or z-slabs of the
     full x-y period; periodic padding in x and y, zero padding at the z
     walls), with its own MFMA forward/backward kernels and Adam;
  3. use: from an LB state the network jumps `every` steps ahead on the whole
     domain; the prediction is lifted back to populations (equilibrium of
     colour densities with the predicted phase field at the pre-jump
     pressure, and the predicted velocity) and the LB step continues for
     `heal` steps, which rebuild the non-equilibrium parts and the interface
     profile;
  4. gate: inside the timed hybrid, an interval of plain LB steps checks the
     network on the current flow: its one-jump prediction over that interval
     must put both fronts within `gate` lattice units of the LB fronts and
     must have a phase-field error at most `skill` times the change of the
     phase field over the interval (the error of keeping the state as it is);
     after a passed check a few jumps follow, then the next LB interval checks
     again.  A plain LB run of the same case is used only afterwards, untimed,
     to state the actual front error of every jump.
"""
from __future__ import annotations

import time

import numpy as np

from . import lbcg as B
from . import surrogate as S
from . import workloads as W


def case(L=64, amp=0.05, g=2e-5, Re=None):
    """Rayleigh-Taylor box [0,L]^2 x [0,4L] (walls at z, periodic sides).  The
    default Reynolds number keeps the kinematic viscosity of the L = 128,
    Re = 1024 case (nu = L sqrt(gL)/Re), so smaller boxes keep its relaxation
    times."""
    Re = 1024.0 * (L / 128.0) ** 1.5 if Re is None else Re
    return W.rayleigh_taylor(L, g=g, amp=amp, Re=Re)


def cs2(p):
    return tuple(0.5 * (1.0 - a) for a in p["alpha"])


def _fields(solver, with_rho=False):
    import torch
    f = solver.fields(0)
    x = torch.stack([f["rhoN"], f["ux"], f["uy"], f["uz"]]).contiguous()
    return (x, (f["rhoR"], f["rhoB"])) if with_rho else x


def snapshots(p, fl, steps, rec, storage="fp32"):
    """LB trajectory: list of (4, N) CUDA float32 (rho^N, u) every `rec` steps
    from step 0 to `steps`, and the wall time of the steps."""
    import torch
    s = B.Solver([(p, fl)], storage=storage)
    out = [_fields(s)]
    wall = 0.0
    try:
        for _ in range(steps // rec):
            torch.cuda.synchronize()
            t0 = time.time()
            s.step(rec)
            torch.cuda.synchronize()
            wall += time.time() - t0
            out.append(_fields(s))
    finally:
        s.close()
    return out, wall


def fronts(rhoN, box):
    """(bubble, spike) interface heights: the first crossing of rho^N = 0 from
    the bottom along the column through the bubble (x = y = 0) and through the
    spike (x = y = L/2), linearly interpolated."""
    nx, ny, nz = box
    col = rhoN.view(nz, ny, nx)
    res = []
    for (x, y) in ((0, 0), (nx // 2, ny // 2)):
        c = col[:, y, x].double().cpu().numpy()
        k = np.nonzero((c[:-1] < 0) & (c[1:] >= 0))[0]
        if k.size == 0:
            res.append(float("nan"))
            continue
        i = int(k[0])
        res.append(i + c[i] / (c[i] - c[i + 1]))
    return tuple(res)


def train(net, trajs, box, lag, iters=400, lr=1e-3, lr_min=1e-5, seed=0, it0=0, total=None, log=None):
    """Adam on (fields_t -> fields_{t+lag snapshots}) pairs drawn at random
    from the trajectories, one pair per batch item, with a cosine learning
    rate from lr to lr_min over `total` iterations (this call runs iterations
    it0 .. it0 + iters - 1 of that schedule); a network shorter than the box in
    z trains on z-slabs that stay inside the box.  Returns the loss history."""
    nz = box[2]
    slab = net.shape[1]
    assert slab <= nz
    total = iters if total is None else total
    rng = np.random.default_rng(seed + it0)
    hist = []
    for k in range(iters):
        it = it0 + k
        for b in range(net.shape[0]):
            tr = trajs[int(rng.integers(len(trajs)))]
            i = int(rng.integers(len(tr) - lag))
            z0 = int(rng.integers(0, nz - slab + 1))
            net.pack(tr[i], box, origin=(0, 0, z0), b=b)
            net.pack(tr[i + lag], box, origin=(0, 0, z0), b=b, target=True)
        net.forward()
        net.mse()
        net.backward()
        net.adam(lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * it / max(1, total - 1))))
        if it % 50 == 0 or k == iters - 1:
            hist.append((it, net.loss[0].item()))
            if log:
                log(f"train it {it} loss {hist[-1][1]:.3e}")
    return hist


def score(hs):
    """Model-selection key of hybrid runs (one network at one number of jumps
    per check) on the validation cases, taken at the worst of them.  Runs
    that all keep every jump and the end within 1 l.u. of the LB fronts beat
    any that do not; among those, the fewest jumps of any case decides (more
    is better), then the largest final error (smaller is better).  Among the
    others the largest final error decides, then the fewest jumps."""
    fins = [float(h["final_front_error"]) for h in hs]
    ok = all(np.isfinite(f) and f <= 1.0 and h["max_jump_error"] <= 1.0 for f, h in zip(fins, hs))
    worst = -max(fins) if all(np.isfinite(f) for f in fins) else -1e9
    jumps = min(h["jumps"] for h in hs)
    return (1, jumps, worst) if ok else (0, worst, jumps)


def full_domain_net(trained, box):
    """A network with the trained weights and buffers for the whole box (z walls: zero padding)."""
    nx, ny, nz = box
    net = S.UNet((1, nz, ny, nx), seed=0, us=trained.us, pmask=3)
    net.load_state(trained.state_dict())
    return net


def predict(net, fields, box):
    import torch
    net.pack(fields, box)
    net.forward()
    out = torch.empty_like(fields)
    net.unpack(out)
    return out


def lift_and_set(solver, pred, p, rho_prev):
    """Equilibrium LB state from the predicted (rho^N, u) at the pressure of
    the state before the jump (sg_lift + lbcg_set_fields)."""
    out = S.lift(pred, cs2(p), rho_prev=rho_prev)
    B.lbcg_set_fields(solver.h, 0, out[0], out[1], out[2], out[3], out[4])


def reference(p, fl, steps, stride):
    """Fronts of the plain LB run every `stride` steps ({t: (bubble, spike)})."""
    box = (p["nx"], p["ny"], p["nz"])
    s = B.Solver([(p, fl)])
    ref = {0: fronts(_fields(s)[0], box)}
    try:
        for t in range(stride, steps + 1, stride):
            s.step(stride)
            ref[t] = fronts(_fields(s)[0], box)
    finally:
        s.close()
    return ref


def lb_time(p, fl, t_start, t_end):
    """Wall time of plain LB steps t_start -> t_end."""
    import torch
    s = B.Solver([(p, fl)])
    try:
        s.step(t_start)
        torch.cuda.synchronize()
        c0 = time.time()
        s.step(t_end - t_start)
        torch.cuda.synchronize()
        return time.time() - c0
    finally:
        s.close()


def front_distance(a, b):
    """Largest distance between the bubble and the spike fronts of two states."""
    return max(abs(a[0] - b[0]), abs(a[1] - b[1]))


def hybrid(net, p, fl, every, t_start, t_end, heal=20, gate=1.0, trust=3, skill=0.5, use_net=True,
           ref_fronts=None):
    """LB to t_start, then the gated hybrid up to t_end, timed as a whole.

    The gate uses only the run's own data.  An interval of `every` plain LB
    steps from state S_a to S_b is also a check: the network predicts S_b from
    S_a; the check passes when the predicted fronts lie within `gate` lattice
    units of the LB fronts and the L2 error of the predicted phase field is at
    most `skill` times |rho^N(S_b) - rho^N(S_a)| (persistence scores exactly 1,
    so a slowly moving front alone does not pass).  After a passed check up to
    `trust` jumps follow (each: predict `every` steps
    ahead, lift the prediction to populations, `heal` LB steps); then another
    LB interval checks again.  A failed check leaves the run on LB intervals,
    each of which is a new check.  With use_net=False the same gate runs with
    persistence (the state left unchanged) in place of the network.

    ref_fronts ({t: fronts} of a plain LB run, optional) is read only outside
    the timed sections, to record the actual front error of every jump for
    evaluation.  Returns the records, the wall time after t_start (checks
    included) and the final front error against ref_fronts (if given)."""
    import torch
    box = (p["nx"], p["ny"], p["nz"])
    s = B.Solver([(p, fl)])
    s.step(t_start)
    torch.cuda.synchronize()
    t, wall, rec, checks, trusted = t_start, 0.0, [], [], 0
    try:
        while t + every <= t_end:
            if trusted > 0 and t + every + heal <= t_end:
                c0 = time.time()
                f, rho = _fields(s, with_rho=True)
                if use_net:
                    lift_and_set(s, predict(net, f, box), p, rho)
                s.step(heal)
                torch.cuda.synchronize()
                wall += time.time() - c0
                t += every + heal
                trusted -= 1
                r = dict(t=t, accepted=True)
                if ref_fronts is not None:
                    r["front_error"] = front_distance(fronts(_fields(s)[0], box), ref_fronts[t])
                rec.append(r)
            else:
                c0 = time.time()
                fa = _fields(s).clone()
                s.step(every)
                fbf = _fields(s)
                pred = predict(net, fa, box) if use_net else fa
                err = front_distance(fronts(pred[0], box), fronts(fbf[0], box))
                moved = float(torch.linalg.vector_norm(fbf[0] - fa[0]))
                rel = float(torch.linalg.vector_norm(pred[0] - fbf[0])) / max(moved, 1e-30)
                torch.cuda.synchronize()
                wall += time.time() - c0
                t += every
                ok = bool(np.isfinite(err) and err <= gate and rel <= skill)
                trusted = trust if ok else 0
                checks.append(dict(t=t, check_error=err, skill=rel, passed=ok))
        c0 = time.time()
        if t < t_end:
            s.step(t_end - t)
        f = _fields(s)
        torch.cuda.synchronize()
        wall += time.time() - c0
        final = front_distance(fronts(f[0], box), ref_fronts[t_end]) if ref_fronts is not None else float("nan")
    finally:
        s.close()
    errs = [r["front_error"] for r in rec if "front_error" in r]
    return dict(records=rec, checks=checks, wall_s=wall, final_front_error=final,
                accepted=len(rec), jumps=len(rec), checks_run=len(checks),
                checks_passed=sum(c["passed"] for c in checks),
                max_jump_error=max(errs) if errs else 0.0,
                jumps_within_gate=sum(1 for e in errs if e <= gate))


def experiment(L=32, every=100, steps=None, train_amps=(0.03, 0.04, 0.06, 0.07), eval_amp=0.05,
               val_amps=(0.045, 0.055),
               iters=3000, segments=6, heal=20, rec=20, batch=4, slab=None, t_start=None, lr=1e-3, lr_min=1e-5,
               gates=(1.0, 0.5), seeds=(7, 8, 9, 10, 11, 12), trusts=(3, 2, 1), skill=0.5, trust_sweep=(), log=None):
    """Train on LB trajectories of train_amps (whole-box inputs, pairs `every`
    steps apart from snapshots every `rec` steps) in `segments` pieces of one
    cosine schedule, once per seed (initial weights and pair sampling); after
    each piece the gated hybrid runs on validation amplitudes (val_amps,
    neither trained on nor evaluated; by default one on each side of
    eval_amp) with each number of jumps per passed check in `trusts`, and the
    weights and trust that are best over all seeds, pieces and trusts by
    `score`, the worst validation case deciding, are kept: the most jumps
    whose drift stays within the gate on both validation cases.  `validated`
    in the summary says whether any candidate did; if none did, a deployment
    keeps plain LB (the hybrid is still measured and reported).  On the
    held-out amplitude eval_amp, run the gated hybrid at each gate, the same
    gate with persistence in place of the network, and the plain LB run; for
    each value in trust_sweep, the hybrid at the first gate with that many
    jumps per passed check.  Returns a summary."""
    import math
    import torch
    steps = steps if steps is not None else int(4.5 * math.sqrt(L / 2e-5)) // every * every
    t_start = t_start if t_start is not None else 5 * every
    assert every % rec == 0
    # the training trajectories stay on the device: (steps/rec + 1) snapshots of
    # 4 FP32 fields per amplitude; refuse a recording interval that cannot fit
    p0, _ = case(L, train_amps[0])
    need = len(train_amps) * (steps // rec + 1) * 4 * 4 * p0["nx"] * p0["ny"] * p0["nz"]
    free, _total = torch.cuda.mem_get_info()
    if need > 0.6 * free:
        raise ValueError(f"training trajectories need {need / 2**30:.0f} GiB of the {free / 2**30:.0f} GiB free; "
                         f"record less often (rec > {rec}) or use fewer amplitudes")
    trajs = []
    gen = 0.0
    for a in train_amps:
        p, fl = case(L, a)
        tr, w = snapshots(p, fl, steps, rec)
        trajs.append(tr)
        gen += w
        if log:
            log(f"trajectory amp {a}: {len(tr)} snapshots, {w:.2f} s")
    stride = math.gcd(every, heal) if heal else every
    vcases = []
    for a in val_amps:
        pv, flv = case(L, a)
        vcases.append((a, pv, flv, reference(pv, flv, steps, stride)))
    p, fl = case(L, eval_amp)
    box = (p["nx"], p["ny"], p["nz"])
    ref = reference(p, fl, steps, stride)
    full = S.UNet((1, p["nz"], p["ny"], p["nx"]), seed=0, us=0.02, pmask=3)
    torch.cuda.synchronize()
    t0 = time.time()
    hist, best, val = [], None, []
    per_seg = max(1, iters // max(1, segments))
    for sd in seeds:
        net = S.UNet((batch, slab or p["nz"], p["ny"], p["nx"]), seed=sd, us=0.02, pmask=3)
        hs = []
        for seg in range(max(1, segments)):
            n_it = per_seg if seg < segments - 1 else iters - per_seg * (segments - 1)
            hs += train(net, trajs, box, every // rec, iters=n_it, lr=lr, lr_min=lr_min, seed=sd, it0=seg * per_seg,
                        total=iters, log=log)
            full.load_state(net.state_dict())
            weights = None
            for tr in trusts:
                hvs = [hybrid(full, pv, flv, every, t_start, steps, heal=heal, gate=1.0, trust=tr, skill=skill,
                              ref_fronts=rv) for _a, pv, flv, rv in vcases]
                key = score(hvs)
                val.append(dict(seed=sd, iters=seg * per_seg + n_it, trust=tr,
                                cases=[dict(amp=a, jumps=hv["jumps"], max_jump_error=hv["max_jump_error"],
                                            final_front_error=hv["final_front_error"])
                                       for (a, *_r), hv in zip(vcases, hvs)]))
                if log:
                    log(f"validation seed {sd} after {val[-1]['iters']} iterations, trust {tr}: " + "; ".join(
                        f"amp {c['amp']}: {c['jumps']} jumps (largest error {c['max_jump_error']:.3f}), final "
                        f"front error {c['final_front_error']:.3f}" for c in val[-1]["cases"]))
                if best is None or key > best[0]:
                    weights = weights if weights is not None else net.state_dict()
                    best = (key, weights, len(val) - 1)
        if not hist or hs[-1][1] < hist[-1][1]:
            hist = hs
    torch.cuda.synchronize()
    train_s = time.time() - t0
    del trajs
    full.load_state(best[1])
    trust = val[best[2]]["trust"]
    # the validation is the gate on using the network at all: the in-run
    # checks bound each jump from the hybrid's own state, not the drift the
    # jumps accumulate, which only a run beside plain LB shows
    validated = best[0][0] == 1
    if log and not validated:
        log("no candidate kept its jumps and its end within 1 l.u. on every validation case: a deployment keeps "
            "plain LB; the hybrid below is measured for the record")
    lb = lb_time(p, fl, t_start, steps)
    res = dict(lattice=[p["nx"], p["ny"], p["nz"]], every=every, steps=steps, t_start=t_start, heal=heal,
               train_amps=list(train_amps), val_amps=list(val_amps), eval_amp=eval_amp, params=net.nparams, train_iters=iters,
               batch=batch, train_shape=list(net.shape), snapshot_every=rec, train_s=train_s, loss_first=hist[0][1], loss_last=min(l for _, l in hist[-5:]),
               seeds=list(seeds), trusts=list(trusts), trust=trust, skill=skill, validation=val, selected_after=val[best[2]]["iters"],
               selected_seed=val[best[2]]["seed"], validated=validated, lb_s=lb, trajectory_s=gen, gates={})
    for g in gates:
        hyb = hybrid(full, p, fl, every, t_start, steps, heal=heal, gate=g, trust=trust, skill=skill, ref_fronts=ref)
        per = hybrid(full, p, fl, every, t_start, steps, heal=heal, gate=g, trust=trust, skill=skill, use_net=False,
                     ref_fronts=ref)
        res["gates"][str(g)] = dict(
            hybrid_s=hyb["wall_s"], gain=lb / hyb["wall_s"], jumps=hyb["jumps"], checks=hyb["checks_run"],
            checks_passed=hyb["checks_passed"], simulated_by_jumps=hyb["jumps"] * (every + heal),
            steps_after_start=steps - t_start, final_front_error=hyb["final_front_error"],
            max_jump_error=hyb["max_jump_error"], jumps_within_gate=hyb["jumps_within_gate"],
            records=[(r["t"], round(r["front_error"], 3)) for r in hyb["records"]],
            check_errors=[(c["t"], round(c["check_error"], 3), round(c["skill"], 3)) for c in hyb["checks"]],
            persistence=dict(jumps=per["jumps"], checks_passed=per["checks_passed"],
                             final_front_error=per["final_front_error"], gain=lb / per["wall_s"]))
        if log:
            log(f"gate {g}: {hyb['jumps']} jumps after {hyb['checks_passed']}/{hyb['checks_run']} passed checks, "
                f"{hyb['jumps_within_gate']} within the gate, largest jump error {hyb['max_jump_error']:.3f}, "
                f"final front error {hyb['final_front_error']:.3f}, gain {lb / hyb['wall_s']:.2f}; persistence "
                f"{per['jumps']} jumps, final {per['final_front_error']:.3f}")
    for tr in trust_sweep:
        h = hybrid(full, p, fl, every, t_start, steps, heal=heal, gate=gates[0], trust=tr, skill=skill, ref_fronts=ref)
        res.setdefault("trust_sweep", {})[str(tr)] = dict(
            gain=lb / h["wall_s"], jumps=h["jumps"], checks=h["checks_run"], checks_passed=h["checks_passed"],
            jumps_within_gate=h["jumps_within_gate"], max_jump_error=h["max_jump_error"],
            final_front_error=h["final_front_error"])
        if log:
            log(f"trust {tr}: {h['jumps']} jumps, {h['jumps_within_gate']} within the gate, final front error "
                f"{h['final_front_error']:.3f}, gain {lb / h['wall_s']:.2f}")
    return res


def bench_summary(rt, gate=1.0):
    """The fields of an experiment() summary that the benchmark reports."""
    g = rt["gates"][str(gate)]
    keep = ("lattice", "every", "heal", "steps", "t_start", "trusts", "trust", "skill", "train_amps", "val_amps", "eval_amp",
            "train_iters", "seeds", "selected_seed", "selected_after", "validated", "train_s", "loss_first", "loss_last",
            "lb_s")
    out = {k: rt[k] for k in keep}
    out.update(gate_lu=gate, **{k: g[k] for k in ("hybrid_s", "gain", "jumps", "checks", "checks_passed",
                                                   "simulated_by_jumps", "steps_after_start", "final_front_error",
                                                   "max_jump_error", "jumps_within_gate", "persistence")})
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Train the surrogate on Rayleigh-Taylor LB runs and measure the "
                                             "gated hybrid against plain LB")
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--heal", type=int, default=20)
    ap.add_argument("--rec", type=int, default=20, help="snapshot interval of the training trajectories")
    ap.add_argument("--slab", type=int, default=0, help="train on z-slabs of this depth (0: whole box)")
    ap.add_argument("--segments", type=int, default=6)
    ap.add_argument("--seeds", default="7,8,9,10,11,12", help="training seeds; the validation picks across all of them")
    ap.add_argument("--trusts", default="3,2,1", help="candidate jumps after each passed check; the validation "
                                                      "picks one with the network")
    ap.add_argument("--skill", type=float, default=0.5, help="largest phase-field error of a passed check, "
                                                            "relative to the change over the interval")
    ap.add_argument("--trust-sweep", default="", help="further jumps-per-check values to evaluate, e.g. 1,2")
    ap.add_argument("--out", default=None, help="write the summary JSON here")
    a = ap.parse_args(argv)
    res = experiment(L=a.L, iters=a.iters, batch=a.batch, lr=a.lr, heal=a.heal, rec=a.rec, slab=a.slab or None,
                     segments=a.segments, seeds=tuple(int(v) for v in a.seeds.split(",")), trusts=tuple(int(v) for v in a.trusts.split(",")),
                     skill=a.skill,
                     trust_sweep=tuple(int(v) for v in a.trust_sweep.split(",") if v), log=lambda m: print(m, flush=True))
    txt = json.dumps(res)
    print(txt, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(json.dumps(res, indent=1) + "\n")


if __name__ == "__main__":
    main()
