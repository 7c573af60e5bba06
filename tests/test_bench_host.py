"""Host-side logic of bench.py (no GPU): the measured-traffic figure comes
from the committed counter summary only while it was taken on the current
beam-kernel sources, the one-GPU contract is enforced, and every profile the
bench reads travels with GPU runs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_traffic_from_committed_summary_matches_sources():
    path = os.path.join(ROOT, "profiles", "beam_kernel_cfg4_fp32_counters.md")
    if not os.path.exists(path):
        pytest.skip("no committed counter summary")
    text = open(path).read()
    if f"`{bench.beam_source_hash()}`" in text:
        t = bench.measured_traffic("cfg4", "fp32")
        assert t is not None and t > 1e9
    else:
        assert bench.measured_traffic("cfg4", "fp32") is None


def test_traffic_absent_for_unprofiled_workloads():
    assert bench.measured_traffic("cfg1", "fp32") is None
    assert bench.measured_traffic("cfg2", "fp8") is None


def test_traffic_ignores_a_summary_of_other_sources(tmp_path, monkeypatch):
    h = bench.beam_source_hash()
    monkeypatch.setattr(bench, "beam_source_hash", lambda: h)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "beam_kernel_cfgx_fp32_counters.md").write_text(
        "- HBM bytes per launch: 123456789012\n- beam sources sha256: `0000000000000000`\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("cfgx", "fp32") is None
    (prof / "beam_kernel_cfgx_fp32_counters.md").write_text(
        f"- HBM bytes per launch: 123456789012\n- beam sources sha256: `{h}`\n")
    assert bench.measured_traffic("cfgx", "fp32") == 123456789012.0


def test_profiles_are_not_excluded_from_gpu_runs():
    path = os.path.join(ROOT, ".gpurunignore")
    if not os.path.exists(path):
        return
    pats = [l.strip() for l in open(path) if l.strip() and not l.startswith("#")]
    assert not any(p.rstrip("/") in ("./profiles", "profiles") for p in pats), pats


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("used_p,dim,want", [
    (64, 768, 32),   # d = 768: doubling is capped and halving leaves six chunks per lane
    (8, 128, 16),    # four chunks per lane: halving would leave eight
    (16, 128, 8),    # two chunks per lane: doubling would leave one
    (16, 96, 8),
    (8, 96, 16),
    (4, 32, 2),
    (1, 4, 1),       # one chunk: nothing else exists
])
def test_counting_launch_lanes(used_p, dim, want):
    got = bench.counting_lanes(used_p, dim)
    assert got == want
    if dim > 4:
        assert got != used_p
