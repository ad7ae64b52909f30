"""The committed measurement artefacts describe the current code: the HBM
traffic figures that the benchmark reports were taken on the same step-kernel
source (a source hash recorded with them), every profile summary names the
command that produced it, and the stored full-size oracle samples were made by
the current oracle."""
import glob
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_profiles_match_the_kernel_source():
    h = bench.kernel_source_hash()
    for storage in ("fp32", "fp16s"):
        path = os.path.join(ROOT, "profiles", f"k_fused_{storage}_rt128x128x512_traffic.json")
        with open(path) as fh:
            d = json.load(fh)
        assert d["kernel_source_sha256_16"] == h, f"{path} was taken on other kernels; profile again"
        assert abs(d["bytes_per_launch"] - d["bytes_per_node"] * d["nodes"]) < 1.0
        assert 0.95 < d["bytes_per_node"] / d["design_bytes_per_node"] < 1.6
        assert all(c.startswith("rocprofv3 --pmc ") for c in d["commands"])


def test_every_summary_names_its_command():
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.txt")):
        with open(path) as fh:
            text = fh.read()
        assert "rocprofv3 " in text, path


def test_full_size_goldens_match_the_oracle_and_inputs():
    """The stored full-size oracle samples were computed by the current oracle
    source; each holds its inputs' digest and its sample of nodes."""
    import hashlib

    import numpy as np

    import full_size_cases as FS
    with open(os.path.join(ROOT, "oracle", "lbcg_oracle.c"), "rb") as fh:
        od = hashlib.sha256(fh.read()).hexdigest()[:16]
    for name, (maker, steps) in FS.CASES.items():
        g = np.load(os.path.join(ROOT, "tests", "golden", name + ".npz"))
        assert str(g["oracle_digest"]) == od, f"{name}: made by another oracle; rerun tests/golden/make_full_size.py"
        assert int(g["steps"]) == steps
        assert g["idx"].size >= 2000 and all(g[k].shape == g["idx"].shape for k in ("rhoN", "ux"))
