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


def write_record(root, launch, source_text=None):
    """A counter record for a workload named c9_test, hashing the step's source as it is."""
    import hashlib
    src = os.path.join(root, "paper_2510_23215_amd", "csrc", "spmm.hip")
    if source_text is not None:
        os.makedirs(os.path.dirname(src), exist_ok=True)
        with open(src, "w") as f:
            f.write(source_text)
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    lines = ["# test record", "source paper_2510_23215_amd/csrc/spmm.hip",
             f"source_sha256_16 {digest}", "bytes_per_chebyshev_step 123456789"]
    lines += [f"{k} {v}" for k, v in launch.items()]
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "spmm_traffic_c9_test.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


LAUNCH = {"chains": 128, "lanes": 6, "schedule": "dynamic", "graphs": "on", "tile": 4,
          "form": "plain", "precision": "fp64", "fused_steps": 0}


def test_traffic_record_matches_only_its_source_and_launch(tmp_path, monkeypatch):
    write_record(str(tmp_path), LAUNCH, "// a filter step\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("c9_test", LAUNCH) == 123456789.0
    assert bench.measured_traffic("c9_test", dict(LAUNCH, lanes=8)) is None
    assert bench.measured_traffic("c9_test", dict(LAUNCH, tile=2)) is None
    assert bench.measured_traffic("c9_missing", LAUNCH) is None


def test_committed_traffic_records_are_complete():
    """Every committed counter record carries the fields bench.py reads: the source it was
    taken on, its hash, the launch keys, and the HBM bytes per Chebyshev step (the library
    counts a fused launch of S steps as S)."""
    import glob
    paths = glob.glob(os.path.join(ROOT, "profiles", "spmm_traffic_*.txt"))
    assert paths
    for path in paths:
        rec = {}
        for line in open(path):
            line = line.strip()
            if line and not line.startswith("#"):
                key, _, val = line.partition(" ")
                rec[key] = val.strip()
        for key in ("source", "source_sha256_16", "bytes_per_chebyshev_step", *LAUNCH):
            assert key in rec, (path, key)
        assert float(rec["bytes_per_chebyshev_step"]) > 0
        assert os.path.isfile(os.path.join(ROOT, rec["source"]))


def test_traffic_record_is_dropped_when_the_step_source_changes(tmp_path, monkeypatch):
    """The record names the hash of the step's source: another source no longer matches."""
    write_record(str(tmp_path), LAUNCH, "// a filter step\n")
    with open(os.path.join(str(tmp_path), "paper_2510_23215_amd", "csrc", "spmm.hip"), "w") as f:
        f.write("// a different filter step\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("c9_test", LAUNCH) is None
