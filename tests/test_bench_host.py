"""Host logic of the benchmark (no GPU): the single-GPU guard and the counter record that
`roofline.traffic` comes from."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def test_traffic_record_matches_only_its_source_and_launch():
    launch = {"chains": 128, "lanes": 6, "schedule": "dynamic", "graphs": "on", "tile": 4,
              "form": "plain", "precision": "fp64"}
    rec = bench.measured_traffic("c2_poisson100", launch)
    assert rec is not None and 1e8 < rec < 3e8
    assert bench.measured_traffic("c2_poisson100", dict(launch, lanes=8)) is None
    assert bench.measured_traffic("c2_poisson100", dict(launch, tile=2)) is None
    assert bench.measured_traffic("c9_missing", launch) is None


def test_traffic_record_is_dropped_when_the_step_source_changes(tmp_path, monkeypatch):
    """A copy of the record pointing at another file: the hash no longer matches."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    text = open(os.path.join(ROOT, "profiles", "spmm_traffic_c2_poisson100.txt")).read()
    (prof / "spmm_traffic_c2_poisson100.txt").write_text(text)
    src = tmp_path / "paper_2510_23215_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "spmm.hip").write_text("// a different filter step\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    launch = {"chains": 128, "lanes": 6, "schedule": "dynamic", "graphs": "on", "tile": 4,
              "form": "plain", "precision": "fp64"}
    assert bench.measured_traffic("c2_poisson100", launch) is None
