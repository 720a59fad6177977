"""bench.py's contract on the CPU: one GPU only, and the traffic figure
reported only while the density kernel is the one the counters measured."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_null_once_the_kernel_source_changes(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    text = open(os.path.join(ROOT, "profiles", "hbm_traffic_two_globules_256.md")).read()
    line = [ln for ln in text.splitlines() if ln.startswith("traffic density_grid_f32")]
    assert len(line) == 1
    assert bench.measured_traffic() is None or bench.measured_traffic() > 0
    # a copy of the tree whose kernel source differs
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "hbm_traffic_two_globules_256.md").write_text(text)
    src = tmp_path / "paper_2208_05524_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "density.hip").write_text("// not the measured kernel\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic() is None
    # the same source as measured gives the recorded figure
    (src / "density.hip").write_bytes(
        open(os.path.join(ROOT, "paper_2208_05524_amd", "csrc", "density.hip"), "rb").read())
    kv = dict(x.split("=", 1) for x in line[0].split()[2:])
    import hashlib
    same = hashlib.sha256((src / "density.hip").read_bytes()).hexdigest() == kv["source_sha256"]
    assert (bench.measured_traffic() == float(kv["bytes_per_launch"])) == same
