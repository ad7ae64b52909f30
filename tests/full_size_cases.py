"""The full-size workloads of the parity tests at benchmark scale: what is
run and for how many steps, and a digest of the generated inputs (so stored
oracle values are only ever compared with runs of the same inputs).  Holds
no arithmetic of the method."""
import hashlib
import json

import numpy as np

from paper_1904_03618_amd import workloads as W

CASES = {
    # Galilean droplet, 128^3 periodic, 500 steps
    "galilean_128_500": (lambda: W.galilean_droplet(128, 20.0, seed=1904), 500),
    # layered channel 64 x 64 x 256, walls on z, density and viscosity ratio 10, force 1e-6
    "channel_64x64x256_ratio10_500": (lambda: W.layered_channel(64, 64, 256, ratio=10.0, visc_ratio=10.0, G=1e-6),
                                      500),
    # Rayleigh-Taylor 128 x 128 x 512 (the benchmark's headline box), 50 steps
    "rayleigh_taylor_128x128x512_50": (lambda: W.rayleigh_taylor(128), 50),
    # droplet impact at the paper's scale, 300 x 300 x 150, Re = 300, 20 steps
    "impact_paper_300x300x150_re300_20": (lambda: W.impact_paper(300.0), 20),
}

NSAMPLE = 2048          # sampled nodes on the interface and in the bulk, each


def input_digest(p, fl):
    h = hashlib.sha256()
    h.update(json.dumps({k: (list(v) if isinstance(v, tuple) else v) for k, v in sorted(p.items())},
                        sort_keys=True, default=str).encode())
    for k in ("rhoR", "rhoB", "ux", "uy", "uz"):
        h.update(np.ascontiguousarray(fl[k], dtype=np.float64).tobytes())
    return h.hexdigest()[:32]


def sample_nodes(rhoN, seed=1):
    """NSAMPLE nodes where the phase field is inside the interface (|rho^N| <
    0.9) and NSAMPLE nodes drawn from the whole box."""
    rng = np.random.default_rng(seed)
    n = rhoN.size
    iface = np.nonzero(np.abs(rhoN) < 0.9)[0]
    a = rng.choice(iface, min(NSAMPLE, iface.size), replace=False) if iface.size else np.empty(0, np.int64)
    b = rng.choice(n, min(NSAMPLE, n), replace=False)
    return np.unique(np.concatenate([a, b])).astype(np.int64)
