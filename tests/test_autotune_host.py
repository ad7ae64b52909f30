"""Host logic of the launch-shape autotuner (no GPU): cache keys, candidate
sets, fused-kernel eligibility and the cached path."""
import json

from paper_1904_03618_amd import autotune as AT
from paper_1904_03618_amd import workloads as W


def _cases():
    return [W.random_state_case(6, 5, 4, seed=1), W.random_state_case(7, 5, 9, seed=2, bc=(0, 0, 1))]


def test_box_class_separates_workloads():
    cases = _cases()
    k = AT.box_class(cases, "fp16s")
    assert k == AT.box_class(cases, "fp16s")
    assert k != AT.box_class(cases, "fp32")
    assert k != AT.box_class(cases[:1], "fp16s")
    assert "moving" not in k
    p, fl = cases[1]
    moving = [cases[0], (dict(p, wall_u=((0.01, 0.0, 0.0), (0.0, 0.0, 0.0))), fl)]
    assert AT.box_class(moving, "fp16s") == k + "|moving=1"


def test_fused_eligibility_and_candidates():
    periodic = [W.random_state_case(6, 5, 4, seed=1)]
    neutral_z = [W.random_state_case(6, 5, 4, seed=1, bc=(0, 0, 1), theta=(90.0, 90.0))]
    wetting_z = [W.random_state_case(6, 5, 4, seed=1, bc=(0, 0, 1), theta=(70.0, 90.0))]
    wall_y = [W.random_state_case(6, 5, 4, seed=1, bc=(0, 1, 0), theta=(90.0, 90.0))]
    p, fl = neutral_z[0]
    moving_z = [(dict(p, wall_u=((0.01, 0.0, 0.0), (0.0, 0.0, 0.0))), fl)]
    assert AT._fused_ok(periodic) and AT._fused_ok(neutral_z)
    assert AT._fused_ok(wetting_z) and AT._fused_ok(moving_z)
    assert not AT._fused_ok(wall_y) and not AT._fused_ok(periodic + wall_y)
    with_f, without = AT.candidates(True), AT.candidates(False)
    assert any(c["kernel"] == "fused" for c in with_f)
    assert all(c["kernel"] == "twopass" for c in without)
    assert len(without) == len({json.dumps(c, sort_keys=True) for c in without})


def test_cached_choice_is_returned_without_timing(tmp_path):
    cases = _cases()
    key = AT.box_class(cases, "bf16s")
    opts = {"kernel": "twopass", "block_nodes": 128, "persistent_blocks": 0, "graph_steps": 8}
    cache = tmp_path / "cache.json"
    cache.write_text(json.dumps({key: {"options": opts}}))
    got, rep = AT.autotune(cases, "bf16s", cache=str(cache))
    assert got == opts and rep["cached"] and rep["key"] == key
