"""Host-side checks of bench.py: the one-GPU guard, the roofline arithmetic
and the bytes each level format is priced at, and the kernel-source hash that
ties counter profiles to the code they were taken on."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bytes_per_node_of_each_level_format():
    # the method's 38 populations read and written, whatever is stored
    assert bench.ALGO_BYTES == {"fp32": 304, "fp16s": 152, "bf16s": 152}
    # pairs: populations plus the writers' densities (8 B) read and written
    assert bench.FUSED_BYTES["pair"] == {"fp32": 320, "fp16s": 168, "bf16s": 168}
    # compact: the rest pair and 18 totals plus 7 FP32 words of writer data
    assert bench.FUSED_BYTES["compact"] == {"fp32": 216, "fp16s": 136, "bf16s": 136}


def test_roofline_prices_the_fused_kernel_at_algorithmic_bytes():
    N = 1000000
    r = bench.roofline({"k_fused": 0.1}, "fp32", N, 0.125, "compact")
    assert abs(r["achieved"] - 304 * N / 1e-4 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    assert abs(r["design_GBps"] - 216 * N / 1e-4 / 1e9) < 1e-6
    assert abs(r["step_achieved"] - 304 * N / 1.25e-4 / 1e9) < 1e-6
    assert r["kernel"] == "k_fused<fp32>" and r["level_format"] == "compact"
    t = bench.roofline({"k_aux": 0.05, "k_collide": 0.1}, "fp16s", N, 0.2)
    assert t["kernel"] == "k_collide<fp16s>" and t["design_GBps"] is None


def test_kernel_source_hash_ignores_comments(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1904_03618_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("kernels.hpp", "d3q19.hpp"):
        shutil.copy(os.path.join(ROOT, "paper_1904_03618_amd", "csrc", f), csrc / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    assert h0 == bench.kernel_source_hash()
    with open(csrc / "kernels.hpp", "a") as fh:
        fh.write("\n// a comment only\n\n")
    assert bench.kernel_source_hash() == h0
    with open(csrc / "kernels.hpp", "a") as fh:
        fh.write("constexpr int kUnused = 1;\n")
    assert bench.kernel_source_hash() != h0
