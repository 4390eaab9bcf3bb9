"""Host-side logic of bench.py (no GPU): the single-GPU guard and the rule
that the measured HBM traffic is reported only for the kernel sources and the
grid the counters were taken on."""
import json
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORD = os.path.join("profiles", "mid_512x512x64_fp32_hbm_traffic.json")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_profiled_grid():
    assert bench.measured_traffic((256, 256, 16)) is None
    assert bench.measured_traffic((512, 512, 32)) is None


def _copy_record_tree(dst):
    with open(os.path.join(ROOT, RECORD)) as f:
        rec = json.load(f)
    os.makedirs(os.path.join(dst, "profiles"))
    shutil.copy(os.path.join(ROOT, RECORD), os.path.join(dst, RECORD))
    for fn in rec["sources"]:
        os.makedirs(os.path.dirname(os.path.join(dst, fn)), exist_ok=True)
        shutil.copy(os.path.join(ROOT, fn), os.path.join(dst, fn))
    return rec


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    rec = _copy_record_tree(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    here = bench.measured_traffic((512, 512, 64))
    if here is not None:
        # counters read the model bytes of one launch within a few per cent
        model = bench.pass_bytes((512, 512, 64), "fp32")["mid"]
        assert 0.9 * model < here < 1.3 * model
        assert here == rec["read_bytes"] + rec["write_bytes"]
    # any edit of a profiled source withdraws the figure
    src = os.path.join(str(tmp_path), rec["sources"][0])
    with open(src, "a") as f:
        f.write("\n")
    assert bench.measured_traffic((512, 512, 64)) is None


def test_traffic_record_without_counters_is_ignored(tmp_path, monkeypatch):
    rec = _copy_record_tree(str(tmp_path))
    for k in ("read_bytes", "write_bytes"):
        rec.pop(k, None)
    with open(os.path.join(str(tmp_path), RECORD), "w") as f:
        json.dump(rec, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic((512, 512, 64)) is None
