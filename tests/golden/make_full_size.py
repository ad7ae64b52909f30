"""Run the FP64 oracle on the full-size workloads of tests/full_size_cases.py
and store its macroscopic fields at sampled nodes (interface and bulk), the
FP64 sums over the box, and digests of the inputs and of the oracle source,
as tests/golden/<name>.npz.  Calls only the oracle and the seeded input
generators; the GPU tests compare the benchmark's launch against these.

  python tests/golden/make_full_size.py [name ...]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402
import full_size_cases as FS  # noqa: E402


def oracle_digest():
    with open(os.path.join(ROOT, "oracle", "lbcg_oracle.c"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def make(name):
    maker, steps = FS.CASES[name]
    p, fl = maker()
    t = time.time()
    f = O.init(p, fl["rhoR"], fl["rhoB"], fl["ux"], fl["uy"], fl["uz"])
    O.run(p, f, steps)
    o = O.fields(p, f)
    del f
    idx = FS.sample_nodes(o["rhoN"])
    out = {k: o[k][idx] for k in ("rhoR", "rhoB", "rhoN", "ux", "uy", "uz")}
    np.savez_compressed(os.path.join(HERE, name + ".npz"), idx=idx, diag=o["diag"], steps=np.int64(steps),
                        input_digest=np.array(FS.input_digest(p, fl)), oracle_digest=np.array(oracle_digest()),
                        **out)
    print(f"{name}: {steps} steps, {idx.size} sampled nodes, {time.time() - t:.0f} s, "
          f"{O.threads()} threads", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(FS.CASES)):
        make(n)
