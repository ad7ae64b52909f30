"""Stated errors of each storage format on the paper's result quantities,
against the FP64 oracle on the same inputs and step counts:
  - the Laplace pressure jump of a static droplet (32^3, density ratio 3,
    radius 8, 1000 steps), relative error;
  - the velocity profile of a layered channel (4 x 4 x 64, viscosity ratio 10,
    10000 steps), maximum error relative to the peak velocity;
  - the bubble and spike fronts of a Rayleigh-Taylor column (16 x 16 x 64,
    amplitude 0.05 L, 2200 steps = 2.5 reference times), in lattice units.
Measured (MI355X): FP32 4e-6 / 2e-6 / 1e-5; FP16S 1.6e-2 / 3.2e-2 / 1.2e-2;
BF16S 1.8e-1 / 2.2e-1 / 0.29.  The bounds below carry about a 2x margin for
the 16-bit forms and keep FP32 at the FP32-parity level."""
import numpy as np
import pytest

import result_metrics as RM
from gpu_helpers import gpu_run, oracle_run
from paper_1904_03618_amd import workloads as W

pytestmark = pytest.mark.gpu

BOUNDS = {  # (laplace relative, channel relative, fronts l.u.)
    "fp32": (1e-4, 1e-4, 1e-3),
    "fp16s": (0.04, 0.07, 0.03),
    "bf16s": (0.35, 0.45, 0.6),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def laplace_case():
    p, _ = W.paper_fluids_droplet(32, 8.0)
    fl = W.droplet_fields(p, (16.3, 15.6, 16.2), 8.0, p["rho_in"])
    o = oracle_run(p, fl, 1000)
    return p, fl, o


@pytest.fixture(scope="module")
def channel_case():
    p, fl = W.layered_channel(4, 4, 64, ratio=1.0, visc_ratio=10.0, G=1e-6)
    return p, fl, oracle_run(p, fl, 10000)


@pytest.fixture(scope="module")
def rt_case():
    from paper_1904_03618_amd import surrogate_rt as R
    p, fl = R.case(16, 0.05)
    return p, fl, oracle_run(p, fl, 2200)


@pytest.mark.parametrize("storage", ["fp32", "fp16s", "bf16s"])
def test_laplace_jump(storage, laplace_case):
    p, fl, o = laplace_case
    inside, outside = o["rhoN"] > 0.99, o["rhoN"] < -0.99
    dpo = RM.laplace_jump(o, p, inside, outside)
    g = gpu_run([(p, fl)], 1000, storage=storage)[0]
    err = abs(RM.laplace_jump(g, p, inside, outside) - dpo) / abs(dpo)
    print("laplace", storage, dpo, err, flush=True)
    assert dpo > 0
    assert err <= BOUNDS[storage][0]


@pytest.mark.parametrize("storage", ["fp32", "fp16s", "bf16s"])
def test_channel_profile(storage, channel_case):
    p, fl, o = channel_case
    uo = RM.channel_profile(o, p)
    ug = RM.channel_profile(gpu_run([(p, fl)], 10000, storage=storage)[0], p)
    err = float(np.abs(ug - uo).max() / np.abs(uo).max())
    print("channel", storage, float(np.abs(uo).max()), err, flush=True)
    assert err <= BOUNDS[storage][1]


@pytest.mark.parametrize("storage", ["fp32", "fp16s", "bf16s"])
def test_rayleigh_taylor_fronts(storage, rt_case):
    p, fl, o = rt_case
    fo = RM.fronts(o["rhoN"], p)
    fg = RM.fronts(gpu_run([(p, fl)], 2200, storage=storage)[0]["rhoN"], p)
    err = max(abs(fg[0] - fo[0]), abs(fg[1] - fo[1]))
    print("fronts", storage, fo, fg, err, flush=True)
    assert np.isfinite(fo).all() and fo[0] > fo[1]       # bubble above spike
    assert err <= BOUNDS[storage][2]
