"""The trained surrogate on a Rayleigh-Taylor run (32 x 32 x 128): trained
on LB snapshots of four perturbation amplitudes by the project's own MFMA
kernels, the weights and the number of jumps per passed check chosen by the
gated hybrid on two validation amplitudes (one on each side of the held-out
one, the worse deciding: the most jumps whose drift stays within the gate),
evaluated on a held-out amplitude as jumps of 100 steps inside the
LB run, gated by checks inside the timed hybrid (the network's one-jump error
on an interval the LB just computed: fronts within the gate and a phase-field
error at most half the change over the interval).  Checks that training
lowers the loss, that some candidate validated (kept its drift within the gate
on both validation amplitudes), that the network passes checks and jumps
where persistence
(the same gate with the state left unchanged) never passes, that most jumps
land within the gate of the plain LB run's fronts and the run ends within 1.5
gates of them; prints the time-to-solution gain over plain LB, checks
included."""
import json

import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_gated_hybrid_on_rayleigh_taylor():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_03618_amd import surrogate_rt as R
    res = R.experiment(L=32, gates=(1.0,), log=lambda m: print(m, flush=True))
    print(json.dumps(res), flush=True)
    g = res["gates"]["1.0"]
    assert res["loss_last"] < 0.5 * res["loss_first"]
    assert res["validated"]
    assert g["jumps"] > 0 and g["checks_passed"] > 0
    assert g["persistence"]["checks_passed"] == 0 and g["persistence"]["jumps"] == 0
    assert g["jumps"] > g["persistence"]["jumps"]
    # the check bounds one jump's error; over 20-30 jumps the errors
    # accumulate (0.01-0.03 l.u. per jump), so the run's end is held to 1.5
    # gates and most single jumps to the gate
    assert g["final_front_error"] <= 1.5
    assert g["jumps_within_gate"] >= 0.8 * g["jumps"]


def test_rejected_jumps_leave_the_lb_run_untouched():
    """The gate as the second fallback: a network with a large random head
    predicts fronts far from the LB run, every check fails, no jump is taken,
    and the hybrid then takes exactly the plain LB steps, so its final fronts
    equal the reference run's bit for bit (front error exactly 0)."""
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_03618_amd import surrogate as S
    from paper_1904_03618_amd import surrogate_rt as R
    p, fl = R.case(16, 0.05)
    every, heal, steps = 100, 20, 1200
    ref = R.reference(p, fl, steps, 20)
    net = S.UNet((1, p["nz"], p["ny"], p["nx"]), seed=3, us=0.02, pmask=3)
    head = net.L["head"]
    rng = np.random.default_rng(5)
    head.w.copy_(torch.tensor(rng.standard_normal(tuple(head.w.shape)).astype(np.float32) * 5.0))
    head.prep()
    h = R.hybrid(net, p, fl, every, 200, steps, heal=heal, gate=1.0, ref_fronts=ref)
    print(h["checks_run"], h["checks_passed"], h["jumps"], h["final_front_error"], flush=True)
    assert h["checks_run"] > 0 and h["checks_passed"] == 0 and h["jumps"] == 0
    assert h["final_front_error"] == 0.0
